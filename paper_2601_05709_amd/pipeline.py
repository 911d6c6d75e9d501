"""One iteration of the compliance hot path through the C ABI.

The steps follow the paper's level-set algorithm (Section "Main algorithm"):
state solve -> compliance and shape derivative -> velocity (descent) solve ->
level-set transport.  Every step is a libfo call on device tensors (the time
step of the update included, fo_time_steps); this file only sequences them.
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import Optional

from . import fo


@dataclass
class IterationOut:
    u: object
    rhs: object
    theta: object
    J: object
    vol: object
    B_tt: object
    dt: float
    state_stats: fo.Stats
    descent_stats: fo.Stats
    times: dict = field(default_factory=dict)


class Iteration:
    """Holds a context and the device buffers of one workload."""

    def __init__(self, w, state_opts: Optional[fo.SolveOpts] = None,
                 descent_opts: Optional[fo.SolveOpts] = None, max_rhs=None, scatter=None):
        import torch
        self.w = w
        dev = torch.device("cuda")
        self.ctx = fo.Context.from_workload(w, max_rhs=max_rhs)
        if scatter is not None:
            self.ctx.set_scatter(scatter)
        self.n_rhs = w.n_rhs
        nd = w.mesh.n_dofs
        self.phi0 = torch.from_numpy(w.phi).to(dev)
        self.phi = self.phi0.clone()
        self.b = torch.from_numpy(w.b.reshape(nd, -1).copy()).to(dev).contiguous()
        self.u = torch.zeros(nd, self.n_rhs, dtype=torch.float64, device=dev)
        self.rhs = torch.zeros(nd, dtype=torch.float64, device=dev)
        self.theta = torch.zeros(nd, dtype=torch.float64, device=dev)
        self.J = torch.zeros(self.n_rhs, dtype=torch.float64, device=dev)
        self.vol = torch.zeros(1, dtype=torch.float64, device=dev)
        self.B_tt = torch.zeros(1, dtype=torch.float64, device=dev)
        self.dopts = fo.DescentOpts(w.alpha, w.gamma_n, w.gamma_s, w.boxes, dim=w.mesh.dim)
        self.state_opts = state_opts or fo.SolveOpts()
        self.descent_opts = descent_opts or fo.SolveOpts()

    def run(self, lambda_vol=0.0, V=1.0, update=True, reset_phi=True, S1=None) -> IterationOut:
        """set_levelset -> state -> derivative -> descent -> (dt, update)."""
        if reset_phi:
            self.phi.copy_(self.phi0)
        c = self.ctx
        c.set_levelset(self.phi)
        st = c.state_solve(self.b, self.u, self.state_opts, n_rhs=self.n_rhs)
        c.shape_derivative(self.u, self.rhs, self.J, self.vol, n_rhs=self.n_rhs,
                           lambda_vol=lambda_vol, V=V, S1=S1)
        ds = c.descent_solve(self.dopts, self.rhs, self.theta, self.descent_opts, self.B_tt)
        dt = 0.0
        if update:
            _, _, dt = fo.time_steps(float(self.B_tt.item()))
            c.levelset_update(self.theta, dt, self.phi)
        return IterationOut(self.u, self.rhs, self.theta, self.J, self.vol, self.B_tt, dt, st, ds)
