"""Oracle of the level-set loop: Algorithm 1 with the Proximal-Perturbed
Lagrangian constraint method (Section "Lagrangian method", eqs. lagrangian,
lag_method, S0andS1), the adaptive time stepping and the stopping criterion
(Section "Other implementation aspects").

TEST INFRASTRUCTURE ONLY: imported by tests/ -- never by the product path.
It shares no code with the HIP library; every step of an iteration calls the
FP64 oracle in oracle.py (assembly, Jacobi-PCG, shape derivative, descent
solve, the paper's transport step).

Readings (where the paper leaves a choice):
* the PPL update runs for iterations i >= 1 (the paper's "i = 1, 2, ..."),
  so iteration 0 uses the initial multipliers (lambda = 0);
* the constraint is the volume fraction C(Omega) = vol(Omega) / V;
* the stopping test runs once per iteration, after the cost and the
  constraint are known and before the derivative, for i > start_to_check;
* no noise in the adaptive time stepping;
* with reinit_step > 0 the transported level set of iteration i is
  reinitialised when i % reinit_step == 0 (the paper's "reinit_step % i = 0"
  read with the operands the other way round, which also covers i = 0).
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import List, Optional

import numpy as np

from .oracle import (adaptive_dt, assemble_descent, assemble_elasticity, element_coef, lame,
                    shape_derivative, transport)
from .reinit import reinit

# the paper's PPL parameters (Section "Lagrangian method")
PPL_R, PPL_DELTA0, PPL_ALPHA, PPL_BETA = 0.999, 0.5, 2000.0, 0.5


@dataclass
class PPL:
    """State (z, lambda, mu, delta) of the constraint method for N_c
    constraints, started at z = lambda = mu = 0, delta = delta0."""
    nc: int = 1
    r: float = PPL_R
    alpha: float = PPL_ALPHA
    beta: float = PPL_BETA
    delta: float = PPL_DELTA0
    z: np.ndarray = None
    lam: np.ndarray = None
    mu: np.ndarray = None

    def __post_init__(self):
        zero = np.zeros(self.nc)
        self.z = zero.copy() if self.z is None else np.asarray(self.z, dtype=np.float64)
        self.lam = zero.copy() if self.lam is None else np.asarray(self.lam, dtype=np.float64)
        self.mu = zero.copy() if self.mu is None else np.asarray(self.mu, dtype=np.float64)

    def update(self, C) -> None:
        """One step of eq. lag_method with the constraint values C(Omega^i):
        mu moves towards lambda by delta (lambda - mu) / (|lambda - mu|^2 + 1),
        lambda = mu + alpha / (1 + alpha beta) (C - 1), z = (lambda - mu) / alpha,
        and delta shrinks by r."""
        C = np.asarray(C, dtype=np.float64)
        d = self.lam - self.mu
        self.mu = self.mu + self.delta * d / (float(d @ d) + 1.0)
        self.lam = self.mu + self.alpha / (1.0 + self.alpha * self.beta) * (C - 1.0)
        self.z = (self.lam - self.mu) / self.alpha
        self.delta = self.r * self.delta

    def lagrangian(self, J: float, C) -> float:
        """eq. lagrangian: J + <lambda, C - 1> + <mu, z> + alpha/2 |z|^2 +
        beta/2 |lambda - mu|^2."""
        C = np.asarray(C, dtype=np.float64)
        d = self.lam - self.mu
        return float(J + self.lam @ (C - 1.0) + self.mu @ self.z + 0.5 * self.alpha * (self.z @ self.z)
                     + 0.5 * self.beta * (d @ d))


def should_stop(i: int, J: List[float], L: Optional[List[float]], C: Optional[List[np.ndarray]],
                start_to_check=30, prev=10, cost_tol=1e-2, lgrn_tol=1e-2, ctrn_tol=1e-2) -> bool:
    """The paper's stopping criterion at iteration i (histories hold the
    values of iterations 0..i).  Without constraints: max over the previous
    `prev` iterates of |J_i - J_j| < cost_tol |J_i|.  With constraints: the
    same on L with lgrn_tol, and max |C_i - 1| < ctrn_tol.  Only for
    i > start_to_check (and only once `prev` earlier values exist)."""
    if i <= start_to_check or i < prev:
        return False
    if C is None:
        Ji = J[i]
        return max(abs(Ji - J[j]) for j in range(i - prev, i)) < cost_tol * abs(Ji)
    Li = L[i]
    lag_ok = max(abs(Li - L[j]) for j in range(i - prev, i)) < lgrn_tol * abs(Li)
    return lag_ok and float(np.max(np.abs(np.asarray(C[i]) - 1.0))) < ctrn_tol


@dataclass
class LoopRecord:
    J: float
    vol: float
    C: float
    L: float
    lam: float
    B_tt: float = float("nan")
    t_end: float = float("nan")
    steps: int = 0
    dt: float = float("nan")


@dataclass
class LoopResult:
    phi: np.ndarray
    records: List[LoopRecord] = field(default_factory=list)
    stopped: bool = False


def optimize(w, n_iter: int, V: Optional[float] = None, smooth: bool = False, dfactor=1e-2,
             t_range=(1e-3, 1e-1), s_range=(8, 16), start_to_check=30, prev=10, cost_tol=1e-2,
             lgrn_tol=1e-2, ctrn_tol=1e-2, rtol=1e-12, reinit_step=0, reinit_pars=(8, 0.1)) -> LoopResult:
    """Algorithm 1 on a fo_inputs.Workload with one load case: per iteration
    the state solve, cost J = b.u and volume, the stopping test, the PPL
    update (V given: constraint vol / V = 1), the descent right-hand side of
    S = S^J + lambda S^C (eq. S0andS1), the velocity solve, the adaptive final
    time and step count (eqs. tend, steps), the paper's transport step of
    phi and, every reinit_step iterations, its reinitialisation.  Returns the
    final phi and one record per iteration."""
    m = w.mesh
    dim = m.dim
    lam_e, mu_e = lame(w.E, w.nu, dim, w.plane_stress)
    Bd = assemble_descent(dim, m.coords, m.conn, m.bfacets, m.bnormal, w.alpha, w.gamma_n, w.gamma_s,
                          w.boxes)
    b = w.b.reshape(-1)
    phi = np.array(w.phi, dtype=np.float64)
    ppl = PPL(1) if V is not None else None
    Vd = 1.0 if V is None else float(V)
    out = LoopResult(phi)
    Js, Ls, Cs = [], [], []
    for i in range(n_iter):
        A_e, chi = element_coef(dim, m.conn, phi, w.ersatz)
        K = assemble_elasticity(dim, m.coords, m.conn, A_e, lam_e, mu_e)
        u, _ = K.solve(b, w.fixed, rtol=rtol)
        _, _, J, vol = shape_derivative(dim, m.coords, m.conn, A_e, chi, lam_e, mu_e, u, 0.0, Vd)
        J = float(J[0])
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
        if should_stop(i, Js, Ls if ppl else None, Cs if ppl else None, start_to_check, prev, cost_tol,
                       lgrn_tol, ctrn_tol):
            out.stopped = True
            break
        rhs, _, _, _ = shape_derivative(dim, m.coords, m.conn, A_e, chi, lam_e, mu_e, u, lam, Vd)
        theta, _ = Bd.solve(rhs, None, rtol=rtol)
        rec.B_tt = float(theta @ rhs)
        rec.t_end, rec.steps, rec.dt = adaptive_dt(rec.B_tt, dfactor, t_range, s_range)
        phi, _ = transport(dim, m.coords, m.conn, theta, rec.dt, rec.steps, phi, smooth=smooth, rtol=rtol)
        if reinit_step and i % reinit_step == 0:
            phi = reinit(dim, m.coords, m.conn, phi, steps=reinit_pars[0], t_end=reinit_pars[1])
    out.phi = phi
    return out
