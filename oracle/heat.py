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


def optimize_heat(w, f, fixed_nodes, n_iter: int, V=None, smooth: bool = False, dfactor=1e-2, t_range=(1e-3, 1e-1),
                  s_range=(8, 16), start_to_check=30, prev=10, cost_tol=1e-2, lgrn_tol=1e-2, ctrn_tol=1e-2,
                  rtol=1e-12, reinit_step=0, reinit_pars=(8, 0.1)):
    """Algorithm 1 on the heat model for the mesh, level set, ersatz value
    and velocity form of the fo_inputs.Workload w, the P1 source f and the
    fixed nodes: per iteration the state, cost and volume, the stopping test,
    the PPL update (V given), the descent right-hand side of S^J + lambda
    S^C, the velocity solve, the adaptive time stepping, the paper's
    transport step and, every reinit_step iterations, the reinitialisation.
    Returns a LoopResult of the oracle loop."""
    from .loop import PPL, LoopRecord, LoopResult, should_stop
    from .oracle import adaptive_dt, assemble_descent, transport
    from .reinit import reinit
    m = w.mesh
    dim = m.dim
    Bd = assemble_descent(dim, m.coords, m.conn, m.bfacets, m.bnormal, w.alpha, w.gamma_n, w.gamma_s, w.boxes)
    phi = np.array(w.phi, dtype=np.float64)
    ppl = PPL(1) if V is not None else None
    Vd = 1.0 if V is None else float(V)
    out = LoopResult(phi)
    Js, Ls, Cs = [], [], []
    for i in range(n_iter):
        u, J, vol, rhs0, A_e, chi = heat_iteration(dim, m.coords, m.conn, phi, f, fixed_nodes, ersatz=w.ersatz,
                                                   lambda_vol=0.0, V=Vd)
        lam = 0.0
        C = vol / Vd
        if ppl is not None:
            if i >= 1:
                ppl.update([C])
            lam = float(ppl.lam[0])
            L = ppl.lagrangian(J, [C])
        else:
            L = J
        rec = LoopRecord(J, vol, C, L, lam)
        out.records.append(rec)
        Js.append(J)
        Ls.append(L)
        Cs.append(np.array([C]))
        if should_stop(i, Js, Ls if ppl else None, Cs if ppl else None, start_to_check, prev, cost_tol, lgrn_tol,
                       ctrn_tol):
            out.stopped = True
            break
        rhs = rhs0 if lam == 0.0 else derivative(dim, m.coords, m.conn, A_e, chi, u, f, lam, Vd)
        theta, _ = Bd.solve(rhs.ravel(), None, rtol=rtol)
        rec.B_tt = float(theta @ rhs.ravel())
        rec.t_end, rec.steps, rec.dt = adaptive_dt(rec.B_tt, dfactor, t_range, s_range)
        phi, _ = transport(dim, m.coords, m.conn, theta, rec.dt, rec.steps, phi, smooth=smooth, rtol=rtol)
        if reinit_step and i % reinit_step == 0:
            phi = reinit(dim, m.coords, m.conn, phi, steps=reinit_pars[0], t_end=reinit_pars[1])
    out.phi = phi
    return out
