"""Oracle of the heat-conduction model (Section "Heat conduction" of the
numerical examples: eqs. heat_cost, heat_prob, heat_AOmega, heat_weak):
minimise J = int A_Omega |grad u|^2 for -div A_Omega grad u = f, u = 0 on
Gamma_0, insulated elsewhere, A_Omega = chi_Omega + 1e-3 chi_(D minus Omega),
under the volume constraint int chi = V.  The adjoint is p = -u, and the
shape derivative has S0 = 2 u grad f, S1 = (2 u f - A |grad u|^2) I +
2 A grad u (x) grad u, plus lambda chi I / V for the constraint.

TEST INFRASTRUCTURE ONLY: imported by tests/ -- never by the product path.
It shares no code with the HIP library.  Element geometry comes from the C
oracle; the element integrals are written out here in numpy and the state is
solved directly (scipy's sparse LU on the free unknowns).

Readings:
* A_Omega per element from the element mean of phi (as for elasticity:
  1 where the mean is negative, the ersatz value otherwise);
* f is a P1 field (nodal values); the load is int f lambda_a = (M f)_a
  with the exact P1 mass matrix, and int u f, int u lambda_a likewise;
* the descent right-hand side follows the elasticity convention:
  rhs_(a,i) = -(int S0_i lambda_a + int (S1 grad lambda_a)_i), so that
  dJ(theta) = -rhs . theta.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from .oracle import element_coef, element_geometry


def _mass_elem(vol, n1):
    return vol[:, None, None] * (np.ones((n1, n1)) + np.eye(n1)) / (n1 * (n1 + 1))


def _assemble(conn, Ke, N):
    n1 = conn.shape[0]
    rows = np.repeat(conn.T, n1, axis=1).ravel()
    cols = np.tile(conn.T, (1, n1)).ravel()
    return sp.csr_matrix((Ke.ravel(), (rows, cols)), shape=(N, N))


def stiffness(dim, coords, conn, A_e):
    """K_ab = sum_e A_e |T_e| grad lambda_a . grad lambda_b."""
    vol, grad = element_geometry(dim, coords, conn)
    Ke = (A_e * vol)[:, None, None] * np.einsum("eai,ebi->eab", grad, grad)
    return _assemble(conn, Ke, coords.shape[0])


def mass(dim, coords, conn):
    """Scalar P1 mass matrix."""
    vol, _ = element_geometry(dim, coords, conn)
    return _assemble(conn, _mass_elem(vol, dim + 1), coords.shape[0])


def solve_state(K, b, fixed_nodes):
    """u with K_ff u_f = b_f on the free nodes, u = 0 on Gamma_0."""
    free = np.asarray(fixed_nodes) == 0
    u = np.zeros(K.shape[0])
    u[free] = spla.spsolve(K[free][:, free].tocsc(), b[free])
    return u


def derivative(dim, coords, conn, A_e, chi, u, f, lambda_vol=0.0, V=1.0):
    """Descent right-hand side [N][dim] of S0 = 2 u grad f and S1 = (2 u f -
    A |grad u|^2) I + 2 A grad u (x) grad u + lambda_vol chi I / V."""
    vol, grad = element_geometry(dim, coords, conn)
    n1 = dim + 1
    Me = _mass_elem(vol, n1)
    ue, fe = u[conn.T], f[conn.T]
    gu = np.einsum("ea,eai->ei", ue, grad)
    gf = np.einsum("ea,eai->ei", fe, grad)
    Mu = np.einsum("eab,eb->ea", Me, ue)                 # int u lambda_a
    uf = np.einsum("ea,ea->e", Mu, fe)                   # int u f
    # int S0_i lambda_a = 2 (grad f)_i int u lambda_a
    s0 = 2.0 * gf[:, None, :] * Mu[:, :, None]
    # int (S1 grad lambda_a)_i
    iso = 2.0 * uf - A_e * vol * np.einsum("ei,ei->e", gu, gu) + lambda_vol * chi * vol / V
    s1 = iso[:, None, None] * grad + 2.0 * (A_e * vol)[:, None, None] * gu[:, None, :] * \
        np.einsum("ei,eai->ea", gu, grad)[:, :, None]
    re = -(s0 + s1)                                      # [E][a][i]
    rhs = np.zeros((coords.shape[0], dim))
    np.add.at(rhs, conn.T.ravel(), re.reshape(-1, dim))
    return rhs


def heat_iteration(dim, coords, conn, phi, f, fixed_nodes, ersatz=1e-3, lambda_vol=0.0, V=1.0):
    """State, cost, volume and descent right-hand side of the heat model for
    the level set phi; returns (u, J, vol, rhs [N][dim], A_e, chi)."""
    coords = np.ascontiguousarray(coords, dtype=np.float64)
    conn = np.ascontiguousarray(conn, dtype=np.int32)
    A_e, chi = element_coef(dim, conn, phi, ersatz)
    K = stiffness(dim, coords, conn, A_e)
    b = mass(dim, coords, conn) @ f
    u = solve_state(K, b, fixed_nodes)
    J = float(u @ (K @ u))
    vol = float((chi * element_geometry(dim, coords, conn)[0]).sum())
    rhs = derivative(dim, coords, conn, A_e, chi, u, f, lambda_vol, V)
    return u, J, vol, rhs, A_e, chi
