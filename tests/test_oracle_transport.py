"""Pins of the oracle's transport step (Section "Transport equation", eqs.
transport, weak_transport, tau_lv) against facts that do not come from the
oracle's closed-form element entries: numerical quadrature of the weak form
on single elements, exact transport of a linear field by a constant velocity,
conservation of the integral under pure diffusion, a sparse direct solver for
the nonsymmetric step systems, and the paper's mesh-size expression."""
import numpy as np
import pytest
import scipy.sparse.linalg as spla

import fo_inputs as fi
import oracle as oc

# degree-2 exact rules on the reference simplex (barycentric points, weights
# summing to 1): edge midpoints in 2D, the symmetric 4-point rule in 3D
_A3 = 0.5854101966249685
_B3 = 0.1381966011250105
RULES = {
    2: (np.array([[0.5, 0.5, 0.0], [0.0, 0.5, 0.5], [0.5, 0.0, 0.5]]), np.full(3, 1.0 / 3.0)),
    3: (np.array([[_A3, _B3, _B3, _B3], [_B3, _A3, _B3, _B3], [_B3, _B3, _A3, _B3],
                  [_B3, _B3, _B3, _A3]]), np.full(4, 0.25)),
}


def quadrature_step_matrix(P, theta_nodes, h2, smooth, dt, sign):
    """Element matrix of eq. weak_transport by quadrature: test lambda_a,
    psi_hat = lambda_a + tau theta . grad lambda_a, trial lambda_b, with
    theta and tau taken at the element mean of the nodal theta."""
    d = P.shape[1]
    n = d + 1
    T = np.hstack([np.ones((n, 1)), P])           # rows [1, x_b]
    C = np.linalg.inv(T)                           # column a: coefficients of lambda_a
    g = C[1:, :].T                                 # g[a] = grad lambda_a
    vol = abs(np.linalg.det(P[1:] - P[0])) / (2 if d == 2 else 6)
    th = theta_nodes.mean(axis=0)
    tau = 0.5 / np.sqrt(1.0 / dt ** 2 + th @ th / h2)
    bary, wts = RULES[d]
    Mt = np.zeros((n, n))
    for lam, wq in zip(bary, wts):
        for a in range(n):
            psi_hat = lam[a] + tau * (th @ g[a])
            for b in range(n):
                phi_b = lam[b]
                adv = 0.5 * (th @ g[b]) * psi_hat
                diff = 0.5 * h2 * (g[b] @ g[a]) if smooth else 0.0  # grad psi_hat = g_a
                Mt[a, b] += wq * vol * (phi_b * psi_hat + sign * dt * (adv + diff))
    return Mt


def one_element_mesh(P):
    d = P.shape[1]
    return np.ascontiguousarray(P, dtype=np.float64), np.arange(d + 1, dtype=np.int32).reshape(d + 1, 1)


@pytest.mark.parametrize("dim", [2, 3])
@pytest.mark.parametrize("smooth", [False, True])
@pytest.mark.parametrize("sign", [1.0, -1.0])
def test_step_matrix_matches_quadrature(dim, smooth, sign):
    rng = np.random.default_rng(40 + dim)
    for trial in range(4):
        P = rng.standard_normal((dim + 1, dim))
        theta = rng.standard_normal((dim + 1, dim))
        h2, dt = 0.3 + rng.random(), 0.05 + 0.2 * rng.random()
        coords, conn = one_element_mesh(P)
        A = oc.assemble_transport(dim, coords, conn, theta.ravel(), h2, smooth, dt, sign).to_scipy().toarray()
        Q = quadrature_step_matrix(P, theta, h2, smooth, dt, sign)
        np.testing.assert_allclose(A, Q, rtol=1e-12, atol=1e-13 * np.abs(Q).max())


@pytest.mark.parametrize("dim", [2, 3])
def test_linear_field_is_transported_exactly(dim):
    """No diffusion, constant theta: phi(x, t) = phi0(x - t theta) is linear
    in x and t, so Crank-Nicolson with the (consistent) Petrov-Galerkin test
    functions reproduces it at the nodes."""
    m = fi.structured_mesh((6, 3) if dim == 2 else (4, 3, 2), (2.0, 1.0) if dim == 2 else (2.0, 1.0, 1.0))
    a = np.array([0.7, -0.4, 0.3][:dim])
    th = np.array([0.25, 0.1, -0.2][:dim])
    phi0 = m.coords @ a + 0.3
    theta = np.tile(th, m.n_nodes)
    dt, steps = 0.04, 5
    phi, its = oc.transport(dim, m.coords, m.conn, theta, dt, steps, phi0, smooth=False, rtol=1e-13)
    expect = phi0 - steps * dt * (a @ th)
    assert its > 0
    np.testing.assert_allclose(phi, expect, rtol=0, atol=1e-11)


@pytest.mark.parametrize("dim", [2, 3])
def test_pure_diffusion_conserves_integral_and_constants(dim):
    m = fi.structured_mesh((8, 4) if dim == 2 else (4, 3, 3), (2.0, 1.0) if dim == 2 else (2.0, 1.0, 1.0))
    rng = np.random.default_rng(7)
    phi0 = rng.standard_normal(m.n_nodes)
    theta = np.zeros(m.n_nodes * dim)
    h2 = oc.transport_h2(dim, m.coords, m.conn)
    phi, _ = oc.transport(dim, m.coords, m.conn, theta, 0.05, 6, phi0, smooth=True, rtol=1e-14)
    # consistent mass: 1^T M (the mass matrix is the theta = 0 step matrix without diffusion)
    M = oc.assemble_transport(dim, m.coords, m.conn, theta, h2, False, 0.05, 1.0).to_scipy()
    w = M.T @ np.ones(m.n_nodes)
    assert abs(w @ phi - w @ phi0) <= 1e-12 * abs(w) @ np.abs(phi0)
    # a constant stays constant
    c, _ = oc.transport(dim, m.coords, m.conn, theta, 0.05, 3, np.full(m.n_nodes, 2.5), smooth=True,
                        rtol=1e-14)
    np.testing.assert_allclose(c, 2.5, rtol=0, atol=1e-12)
    # without velocity the step matrix is symmetric
    L = oc.assemble_transport(dim, m.coords, m.conn, theta, h2, True, 0.05, 1.0).to_scipy()
    assert abs(L - L.T).max() < 1e-15 * abs(L).max()


@pytest.mark.parametrize("dim", [2, 3])
def test_bicgstab_matches_direct_solve_and_step_uses_it(dim):
    m = fi.structured_mesh((10, 5) if dim == 2 else (5, 3, 3), (2.0, 1.0) if dim == 2 else (2.0, 1.0, 1.0))
    rng = np.random.default_rng(11)
    theta = rng.standard_normal(m.n_nodes * dim) * 3.0
    phi0 = rng.standard_normal(m.n_nodes)
    h2 = oc.transport_h2(dim, m.coords, m.conn)
    dt = 0.02
    L = oc.assemble_transport(dim, m.coords, m.conn, theta, h2, True, dt, 1.0)
    R = oc.assemble_transport(dim, m.coords, m.conn, theta, h2, True, dt, -1.0)
    Ls = L.to_scipy()
    assert abs(Ls - Ls.T).max() > 1e-6  # nonsymmetric
    b = R.matvec(phi0)
    x_ref = spla.spsolve(Ls.tocsc(), b)
    x, info = oc.bicgstab(L, b, phi0, rtol=1e-13)
    assert info.status == 0
    assert np.linalg.norm(x - x_ref) <= 1e-11 * np.linalg.norm(x_ref)
    # two steps of the oracle equal two direct solves
    p1 = spla.spsolve(Ls.tocsc(), R.matvec(phi0))
    p2 = spla.spsolve(Ls.tocsc(), R.matvec(p1))
    phi, _ = oc.transport(dim, m.coords, m.conn, theta, dt, 2, phi0, smooth=True, h2=h2, rtol=1e-13)
    assert np.linalg.norm(phi - p2) <= 1e-10 * np.linalg.norm(p2)


def test_no_velocity_no_diffusion_is_identity():
    m = fi.structured_mesh((6, 3), (2.0, 1.0))
    phi0 = np.random.default_rng(3).standard_normal(m.n_nodes)
    phi, _ = oc.transport(2, m.coords, m.conn, np.zeros(2 * m.n_nodes), 0.1, 4, phi0, smooth=False,
                          rtol=1e-14)
    np.testing.assert_allclose(phi, phi0, rtol=0, atol=1e-13)


@pytest.mark.parametrize("dim", [2, 3])
def test_h2_is_the_papers_mesh_size_expression(dim):
    cells = (8, 4) if dim == 2 else (4, 2, 2)
    m = fi.structured_mesh(cells, (2.0, 1.0) if dim == 2 else (2.0, 1.0, 1.0))
    NT = m.conn.shape[1]
    vol_D = 2.0
    expect = 4 * vol_D / (NT * np.sqrt(3)) if dim == 2 else (6 * np.sqrt(2) * vol_D / NT) ** (2.0 / 3.0)
    assert oc.transport_h2(dim, m.coords, m.conn) == pytest.approx(expect, rel=1e-14)
    # for a regular tetrahedron / equilateral triangle of edge a it equals a^2
    a = 0.7
    if dim == 2:
        P = np.array([[0, 0], [a, 0], [a / 2, a * np.sqrt(3) / 2]])
    else:
        P = np.array([[1, 1, 1], [1, -1, -1], [-1, 1, -1], [-1, -1, 1]], dtype=float) * a / (2 * np.sqrt(2))
    coords, conn = one_element_mesh(P)
    assert oc.transport_h2(dim, coords, conn) == pytest.approx(a * a, rel=1e-12)
