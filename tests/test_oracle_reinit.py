"""Pins of the oracle's reinitialisation (Section "Other implementation
aspects", eqs. Eikonal, HJ, grad_H, weak_HJ) against facts that do not come
from its closed-form element integrals: numerical quadrature of the weak
form on single elements (Euler and Adams-Bashforth steps), the exact
solution for a constant level set, a direct solve of the paper's scheme, and
the effect the equation has on a steep interface."""
import numpy as np
import pytest

import fo_inputs as fi
from oracle import element_geometry, transport_h2
from oracle import reinit as orr

_A3, _B3 = 0.5854101966249685, 0.1381966011250105
RULES = {
    2: (np.array([[0.5, 0.5, 0.0], [0.0, 0.5, 0.5], [0.5, 0.0, 0.5]]), np.full(3, 1.0 / 3.0)),
    3: (np.array([[_A3, _B3, _B3, _B3], [_B3, _A3, _B3, _B3], [_B3, _B3, _A3, _B3],
                  [_B3, _B3, _B3, _A3]]), np.full(4, 0.25)),
}


def quadrature_system(P, u, v, S_nodes, h2, dt):
    """One step's element matrix and vector by quadrature of eq. weak_HJ on
    the element P, with S at the element mean (the oracle's reading)."""
    d = P.shape[1]
    n = d + 1
    T = np.hstack([np.ones((n, 1)), P])
    Cf = np.linalg.inv(T)
    g = Cf[1:, :].T                                   # g[a] = grad lambda_a
    vol = abs(np.linalg.det(P[1:] - P[0])) / (2 if d == 2 else 6)
    S = S_nodes.mean()
    gu = g.T @ u
    gv = None if v is None else g.T @ v
    nu = np.linalg.norm(gu)
    gH = S * gu / nu if nu > 0 else np.zeros(d)
    tau = 0.5 / np.sqrt(1 / dt ** 2 + S * S / h2)
    H = lambda p: S * np.linalg.norm(p)
    bary, wts = RULES[d]
    A = np.zeros((n, n))
    r = np.zeros(n)
    for lam, wq in zip(bary, wts):
        uq = lam @ u
        for a in range(n):
            psi_hat = lam[a] + tau * (gH @ g[a])
            grad_psi_hat = g[a]
            if v is None:
                G = -H(gu) * psi_hat - h2 * (gu @ grad_psi_hat)
            else:
                G = 0.5 * (H(gv) - 3 * H(gu)) * psi_hat + h2 * 0.5 * ((gv - 3 * gu) @ grad_psi_hat)
            r[a] += wq * vol * ((uq + dt * S) * psi_hat + dt * G)
            for b in range(n):
                A[a, b] += wq * vol * lam[b] * psi_hat
    return A, r


@pytest.mark.parametrize("dim", [2, 3])
@pytest.mark.parametrize("euler", [True, False])
def test_step_system_matches_quadrature(dim, euler):
    rng = np.random.default_rng(60 + dim + 2 * euler)
    for trial in range(4):
        P = rng.standard_normal((dim + 1, dim))
        conn = np.arange(dim + 1, dtype=np.int32).reshape(dim + 1, 1)
        u = rng.standard_normal(dim + 1)
        v = None if euler else rng.standard_normal(dim + 1)
        S_nodes = rng.uniform(-0.9, 0.9, dim + 1)
        h2, dt = 0.2 + rng.random(), 0.01 + 0.05 * rng.random()
        vol, grad = element_geometry(dim, np.ascontiguousarray(P), conn)
        A, r = orr.step_system(dim, conn, vol, grad, np.array([S_nodes.mean()]), h2, dt, u, v)
        Aq, rq = quadrature_system(P, u, v, S_nodes, h2, dt)
        np.testing.assert_allclose(A.toarray(), Aq, rtol=1e-12, atol=1e-13 * np.abs(Aq).max())
        np.testing.assert_allclose(r, rq, rtol=1e-12, atol=1e-13 * np.abs(rq).max())


@pytest.mark.parametrize("dim", [2, 3])
def test_constant_level_set_moves_at_rate_S(dim):
    """grad varphi = 0: H = 0 and no diffusion, so varphi(t) = c + t S(c)
    exactly, for the Euler step and the Adams-Bashforth steps alike."""
    m = fi.structured_mesh((6, 3) if dim == 2 else (3, 2, 2), (2.0, 1.0) if dim == 2 else (2.0, 1.0, 1.0))
    h2 = transport_h2(dim, m.coords, m.conn)
    for c in (0.3, -0.05):
        out = orr.reinit(dim, m.coords, m.conn, np.full(m.n_nodes, c), steps=8, t_end=0.1)
        np.testing.assert_allclose(out, c + 0.1 * c / np.sqrt(c * c + h2), rtol=0, atol=1e-13)


def test_steep_interface_relaxes_towards_unit_slope():
    """phi = 3 (x - 1): the equation drives |grad varphi| towards 1 (S(1 -
    |grad varphi|) < 0 on the positive side, > 0 on the negative side) while
    the zero level set stays at x = 1."""
    m = fi.structured_mesh((40, 10), (2.0, 1.0))
    phi = 3.0 * (m.coords[:, 0] - 1.0)
    out = orr.reinit(2, m.coords, m.conn, phi, steps=8, t_end=0.1)
    vol, grad = element_geometry(2, m.coords, m.conn)
    g0 = np.linalg.norm(np.einsum("ea,eai->ei", phi[m.conn.T], grad), axis=1)
    g1 = np.linalg.norm(np.einsum("ea,eai->ei", out[m.conn.T], grad), axis=1)
    xc = m.coords[m.conn.T, 0].mean(axis=1)
    near = np.abs(xc - 1.0) < 0.3
    assert np.all(g0[near] == pytest.approx(3.0))
    assert g1[near].mean() < 2.9 and g1[near].min() > 1.0
    # the crossing on the line y = 0.5 stays within a tenth of a cell of x = 1
    row = np.isclose(m.coords[:, 1], 0.5)
    x, f = m.coords[row, 0], out[row]
    o = np.argsort(x)
    x, f = x[o], f[o]
    k = np.nonzero(np.sign(f[:-1]) != np.sign(f[1:]))[0][0]
    xz = x[k] - f[k] * (x[k + 1] - x[k]) / (f[k + 1] - f[k])
    assert abs(xz - 1.0) < 0.1 * (2.0 / 40)
