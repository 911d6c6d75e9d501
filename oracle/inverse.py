"""Oracle of the inverse elasticity problem (Section "Inverse problem" of the
model problem: eqs. cost, f-prob, g-prob, AOmega, w-f, w-g, the adjoint
problems of eqs. dL1, dL2 and the shape derivative of eq. SDelast_inv), for
one force-displacement pair (f, g):

    J = alpha/2 int |u - v - g|^2 + beta/2 int_Gamma1 |u - g|^2,

u the f-problem (u = 0 on Gamma_0, traction f on Gamma_1), y = v + g the
g-problem (v = 0 on the whole boundary), A_Omega = kappa chi + 1 otherwise,
the adjoints p (Gamma_0 clamped) and q (whole boundary clamped), and
S0 = -alpha Dg^T (u - v - g) + A sum_ij sigma(q)_ij grad eps(g)_ij,
S1 = [alpha/2 |u - v - g|^2 + A (sigma(u):eps(p) + sigma(v+g):eps(q))] I
     - A (Du^T sigma(p) + Dp^T sigma(u)) - A (Dv^T sigma(q) + Dq^T sigma(v+g)).

TEST INFRASTRUCTURE ONLY: imported by tests/ -- never by the product path.
It shares no code with the HIP library.  Stiffness matrices come from the C
oracle; the mass matrices and the element integrals of the derivative are
written out here in numpy; the states are solved directly (scipy's sparse LU
on the free unknowns).

Readings:
* A_Omega per element from the element mean of phi: kappa where it is
  negative, 1 elsewhere (the paper's implementation takes kappa where phi < 0);
* g is a P1 field on the whole domain that vanishes on Gamma_0 (its
  Dirichlet extension); eps(g) is constant on each element, so the term
  A sigma(q)_ij grad eps(g)_ij of S0 vanishes element by element;
* the velocity lives in H^1_0 (theta = 0 on the whole boundary, so that T_t
  is the identity on Gamma_1): the velocity solve clamps every boundary
  unknown;
* Du is the Jacobian (Du)_ij = d_j u_i; S1 : D theta = sum_ij S1_ij d_j theta_i,
  and the descent right-hand side is rhs_(a,i) = -(int S0_i lambda_a +
  int (S1 grad lambda_a)_i), as for the compliance.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from .loop import LoopRecord, LoopResult, should_stop
from .oracle import adaptive_dt, assemble_descent, assemble_elasticity, element_geometry, lame, transport
from .reinit import reinit


def element_kappa(conn, phi, kappa):
    """A_e = kappa where the element mean of phi is negative, else 1; chi."""
    chi = (phi[conn.T].mean(axis=1) < 0.0).astype(np.float64)
    return np.where(chi > 0, kappa, 1.0), chi


def vector_mass(dim, coords, conn):
    """P1 mass matrix for d-vector fields (DOF a*d + i)."""
    vol, _ = element_geometry(dim, coords, conn)
    n1 = dim + 1
    Me = vol[:, None, None] * (np.ones((n1, n1)) + np.eye(n1)) / (n1 * (n1 + 1))
    rows, cols, vals = [], [], []
    for i in range(dim):
        rows.append(np.repeat(conn.T, n1, axis=1).ravel() * dim + i)
        cols.append(np.tile(conn.T, (1, n1)).ravel() * dim + i)
        vals.append(Me.ravel())
    N = coords.shape[0] * dim
    return sp.csr_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))), shape=(N, N))


def facet_mass(dim, coords, facets):
    """P1 mass on the boundary facets [d][F] (Gamma_1) for d-vector fields:
    |F| (1 + delta_ab) / (d (d + 1)) per facet."""
    P = coords[facets.T]                                  # [F][d][d]
    if dim == 2:
        area = np.linalg.norm(P[:, 1] - P[:, 0], axis=1)
    else:
        area = 0.5 * np.linalg.norm(np.cross(P[:, 1] - P[:, 0], P[:, 2] - P[:, 0]), axis=1)
    Mf = area[:, None, None] * (np.ones((dim, dim)) + np.eye(dim)) / (dim * (dim + 1))
    rows, cols, vals = [], [], []
    for i in range(dim):
        rows.append(np.repeat(facets.T, dim, axis=1).ravel() * dim + i)
        cols.append(np.tile(facets.T, (1, dim)).ravel() * dim + i)
        vals.append(Mf.ravel())
    N = coords.shape[0] * dim
    return sp.csr_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))), shape=(N, N))


def _solve(K, b, fixed):
    free = np.asarray(fixed) == 0
    x = np.zeros(K.shape[0])
    x[free] = spla.spsolve(K[free][:, free].tocsc(), b[free])
    return x


def _jac(F, conn, grad, dim):
    """Element Jacobians (DF)_ij = d_j F_i of the P1 vector field F: [E][d][d]."""
    Fe = F.reshape(-1, dim)[conn.T]                       # [E][a][i]
    return np.einsum("eai,eaj->eij", Fe, grad)


def _sigma(D, lam, mu):
    eps = 0.5 * (D + np.transpose(D, (0, 2, 1)))
    tr = np.trace(eps, axis1=1, axis2=2)
    return lam * tr[:, None, None] * np.eye(D.shape[1]) + 2.0 * mu * eps, eps


def derivative(dim, coords, conn, A_e, lam, mu, u, v, p, q, g, alpha):
    """Descent right-hand side [N*d] of eq. SDelast_inv (S0, S1 above)."""
    vol, grad = element_geometry(dim, coords, conn)
    n1 = dim + 1
    Me = vol[:, None, None] * (np.ones((n1, n1)) + np.eye(n1)) / (n1 * (n1 + 1))
    Du, Dv, Dp, Dq, Dg = (_jac(F, conn, grad, dim) for F in (u, v, p, q, g))
    su, eu = _sigma(Du, lam, mu)
    sp_, ep = _sigma(Dp, lam, mu)
    sq, eq = _sigma(Dq, lam, mu)
    svg, _ = _sigma(Dv + Dg, lam, mu)
    w = (u - v - g).reshape(-1, dim)[conn.T]              # [E][a][i]
    Mw = np.einsum("eab,ebi->eai", Me, w)                 # int w lambda_a
    ww = np.einsum("eai,eai->e", Mw, w)                   # int |w|^2
    iso = 0.5 * alpha * ww + A_e * vol * (np.einsum("eij,eij->e", su, ep) + np.einsum("eij,eij->e", svg, eq))
    tt = lambda D, S: np.einsum("eki,ekj->eij", D, S)     # D^T S
    T = (A_e * vol)[:, None, None] * (tt(Du, sp_) + tt(Dp, su) + tt(Dv, sq) + tt(Dq, svg))
    # int (S1 grad lambda_a)_i = iso d_i lambda_a - sum_j T_ij d_j lambda_a
    s1 = iso[:, None, None] * grad - np.einsum("eij,eaj->eai", T, grad)
    # int S0_i lambda_a = -alpha sum_k (Dg)_ki int w_k lambda_a
    s0 = -alpha * np.einsum("eki,eak->eai", Dg, Mw)
    re = -(s0 + s1)
    rhs = np.zeros((coords.shape[0], dim))
    np.add.at(rhs, conn.T.ravel(), re.reshape(-1, dim))
    return rhs.ravel()


def cost(M, MG, u, v, g, alpha, beta):
    w = u - v - g
    z = u - g
    return 0.5 * alpha * float(w @ (M @ w)) + 0.5 * beta * float(z @ (MG @ z))


def inverse_iteration(wi, phi=None, X=None):
    """States u, v, adjoints p, q, cost J and the descent right-hand side of
    the inverse problem for the InverseWorkload wi (X: node coordinates,
    default the mesh's).  Returns a dict."""
    m = wi.mesh
    dim = m.dim
    X = m.coords if X is None else X
    phi = wi.phi if phi is None else phi
    lam, mu = lame(wi.E, wi.nu, dim, wi.plane_stress)
    A_e, chi = element_kappa(m.conn, phi, wi.kappa)
    K = assemble_elasticity(dim, X, m.conn, A_e, lam, mu).to_scipy()
    M = vector_mass(dim, X, m.conn)
    MG = facet_mass(dim, X, m.bfacets)
    g = wi.g
    u = _solve(K, wi.f, wi.fixed0)
    v = _solve(K, -(K @ g), wi.fixed_all)
    w = u - v - g
    p = _solve(K, -wi.alpha * (M @ w) - wi.beta * (MG @ (u - g)), wi.fixed0)
    q = _solve(K, wi.alpha * (M @ w), wi.fixed_all)
    J = cost(M, MG, u, v, g, wi.alpha, wi.beta)
    rhs = derivative(dim, X, m.conn, A_e, lam, mu, u, v, p, q, g, wi.alpha)
    return dict(u=u, v=v, p=p, q=q, J=J, rhs=rhs, A_e=A_e, chi=chi, K=K, M=M, MG=MG)


def velocity(wi, rhs, alpha_v=0.01, rtol=1e-12):
    """theta in H^1_0: the descent form (alpha_v mass + gradient terms, no
    boundary or subdomain penalty) with every boundary unknown clamped."""
    m = wi.mesh
    Bd = assemble_descent(m.dim, m.coords, m.conn, m.bfacets, m.bnormal, alpha_v, 0.0, 0.0, None)
    theta, info = Bd.solve(np.where(wi.fixed_all == 1, 0.0, rhs), wi.fixed_all, rtol=rtol)
    return theta, info


def pairs_iteration(wi, phi):
    """Cost and descent right-hand side summed over the workload's pairs (in
    pair order) for the level set phi."""
    J, rhs = 0.0, None
    for k in range(wi.n_pairs):
        r = inverse_iteration(wi.pair(k), phi=phi)
        J += r["J"]
        rhs = r["rhs"] if rhs is None else rhs + r["rhs"]
    return J, rhs


def optimize_inverse(wi, n_iter: int, smooth: bool = False, dfactor=1e-2, t_range=(1e-3, 1e-1), s_range=(8, 16),
                     start_to_check=30, prev=10, cost_tol=1e-2, alpha_v=0.01, rtol=1e-12, reinit_step=0,
                     reinit_pars=(8, 0.1)) -> LoopResult:
    """Algorithm 1 on the inverse problem (no constraint): per iteration the
    states and adjoints of every pair, the summed cost, the stopping test on
    the cost, the summed descent right-hand side, the H^1_0 velocity, the
    adaptive final time and step count (eqs. tend, steps), the paper's
    transport step and, every reinit_step iterations, the reinitialisation.
    Records carry J (= L) and the time stepping; vol and C are 0."""
    m = wi.mesh
    phi = np.array(wi.phi, dtype=np.float64)
    out = LoopResult(phi)
    Js = []
    for i in range(n_iter):
        J, rhs = pairs_iteration(wi, phi)
        rec = LoopRecord(J, 0.0, 0.0, J, 0.0)
        out.records.append(rec)
        Js.append(J)
        if should_stop(i, Js, None, None, start_to_check, prev, cost_tol):
            out.stopped = True
            break
        theta, _ = velocity(wi, rhs, alpha_v=alpha_v, rtol=rtol)
        rec.B_tt = float(theta @ rhs)
        rec.t_end, rec.steps, rec.dt = adaptive_dt(rec.B_tt, dfactor, t_range, s_range)
        phi, _ = transport(m.dim, m.coords, m.conn, theta, rec.dt, rec.steps, phi, smooth=smooth, rtol=rtol)
        if reinit_step and i % reinit_step == 0:
            phi = reinit(m.dim, m.coords, m.conn, phi, steps=reinit_pars[0], t_end=reinit_pars[1])
    out.phi = phi
    return out
