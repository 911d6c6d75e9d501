"""Oracle of the reinitialisation of the level set (Section "Other
implementation aspects": the diffusive Eikonal equation, eqs. Eikonal, HJ,
grad_H and weak_HJ): pseudo-time steps of

    d/dt varphi + H(grad varphi) = S(phi) + h^2 lap varphi,   H(p) = S(phi) |p|,

from varphi(0) = phi, with Petrov-Galerkin test functions psi_hat = psi +
tau grad H(grad varphi(t)) . grad psi, explicit Euler for the first step and
two-step Adams-Bashforth after it.

TEST INFRASTRUCTURE ONLY: imported by tests/ -- never by the product path.
It shares no code with the HIP library.  Element geometry comes from the C
oracle, the element integrals are written out here in numpy, and each step's
sparse system is solved directly (scipy's sparse LU).

Readings (where the paper leaves a choice):
* S(phi) = phi / sqrt(phi^2 + h^2) enters per element at the mean of its
  nodal values (a one-point rule, as theta in the transport step); h^2 is
  the paper's mesh-size expression (as in the transport step);
* grad H on an element is S_e g / |g| with g the element gradient of
  varphi(t), and tau_e = 1/2 (dt^-2 + S_e^2 / h^2)^(-1/2).  p / |p| has no
  limit at p = 0, and an element whose vertex values agree (a symmetric
  extremum of the level set) has a gradient of pure rounding, pointing
  anywhere: grad H is taken as 0 where max_a u_a - min_a u_a <= 1e-12
  max_a |u_a| (and where g = 0);
* the paper's defaults: 8 steps up to pseudo-time 0.1.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from .oracle import element_geometry, transport_h2


def _elem_grad(u, conn, grad):
    """Element gradients of the P1 field u: [E][d]."""
    return np.einsum("ea,eai->ei", u[conn.T], grad)


def step_system(dim, conn, vol, grad, Sbar, h2, dt, u, v=None):
    """Matrix and right-hand side of one step of eq. weak_HJ from varphi(t) = u
    and varphi(t - dt) = v (v None: the explicit Euler first step).  Returns
    (scipy CSR matrix, rhs)."""
    N = u.shape[0]
    n1 = dim + 1
    E = conn.shape[1]
    gu = _elem_grad(u, conn, grad)
    nu = np.linalg.norm(gu, axis=1)
    ue0 = u[conn.T]
    flat = (ue0.max(axis=1) - ue0.min(axis=1) <= 1e-12 * np.abs(ue0).max(axis=1)) | (nu == 0)
    dirn = np.where(flat[:, None], 0.0, gu / np.where(flat, 1.0, nu)[:, None])
    gH = Sbar[:, None] * dirn                                   # grad H per element
    tau = 0.5 / np.sqrt(1.0 / dt ** 2 + Sbar ** 2 / h2)
    tg = np.einsum("ei,eai->ea", gH, grad)                      # grad H . grad lambda_a
    # P1 mass: |T| (1 + delta_ab) / ((d+1)(d+2))
    Me = vol[:, None, None] * (np.ones((n1, n1)) + np.eye(n1)) / (n1 * (n1 + 1))
    # int lambda_b psi_hat_a = M_ab + tau (grad H . grad lambda_a) |T| / (d+1)
    Le = Me + (tau[:, None] * tg * vol[:, None] / n1)[:, :, None]
    ue = u[conn.T]
    ubar = ue.mean(axis=1)
    ones_hat = vol[:, None] / n1 + tau[:, None] * tg * vol[:, None]   # int psi_hat_a
    if v is None:
        c = -Sbar * nu                                           # -H(grad u)
        dvec = -gu                                               # -grad u
    else:
        gv = _elem_grad(v, conn, grad)
        c = 0.5 * Sbar * (np.linalg.norm(gv, axis=1) - 3.0 * nu)  # (H(grad v) - 3 H(grad u)) / 2
        dvec = 0.5 * (gv - 3.0 * gu)                              # (grad v - 3 grad u) / 2
    re = (np.einsum("eab,eb->ea", Me, ue) + tau[:, None] * tg * (vol * ubar)[:, None]   # int u psi_hat
          + dt * Sbar[:, None] * ones_hat                                               # int dt S psi_hat
          + dt * c[:, None] * ones_hat                                                  # dt G, transport part
          + dt * h2 * vol[:, None] * np.einsum("ei,eai->ea", dvec, grad))               # dt G, diffusion part
    rows = np.repeat(conn.T, n1, axis=1).ravel()
    cols = np.tile(conn.T, (1, n1)).ravel()
    A = sp.csr_matrix((Le.ravel(), (rows, cols)), shape=(N, N))
    rhs = np.zeros(N)
    np.add.at(rhs, conn.T.ravel(), re.ravel())
    return A, rhs


def s_of_phi(phi, h2):
    """S(phi) = phi / sqrt(phi^2 + h^2) at the nodes."""
    return phi / np.sqrt(phi * phi + h2)


def reinit(dim, coords, conn, phi, steps=8, t_end=0.1, h2=None):
    """`steps` pseudo-time steps of eq. weak_HJ up to t_end from phi; returns
    varphi(t_end)."""
    coords = np.ascontiguousarray(coords, dtype=np.float64)
    conn = np.ascontiguousarray(conn, dtype=np.int32)
    if h2 is None:
        h2 = transport_h2(dim, coords, conn)
    vol, grad = element_geometry(dim, coords, conn)
    phi = np.asarray(phi, dtype=np.float64)
    Sbar = s_of_phi(phi, h2)[conn.T].mean(axis=1)
    dt = t_end / steps
    u, v = phi.copy(), None
    for _ in range(steps):
        A, rhs = step_system(dim, conn, vol, grad, Sbar, h2, dt, u, v)
        x = spla.spsolve(A.tocsc(), rhs)
        v, u = u, x
    return u
