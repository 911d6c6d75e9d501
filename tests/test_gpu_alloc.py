"""After fo_create, the per-iteration calls allocate no device memory: level
set, state solves (FP64 and FP32 + refinement), shape derivative, velocity
solve, level-set update, transport, reinitialisation and the heat model's
calls leave the library's allocation count unchanged."""
import numpy as np
import pytest

import fo_inputs as fi

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from paper_2601_05709_amd import fo  # noqa: E402


def dev(a, dtype=np.float64):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=dtype)).cuda()


@pytest.mark.parametrize("name", ["2d_32x16", "3d_8x4x4"])
def test_iteration_calls_allocate_nothing(name):
    w = fi.cantilever_2d((32, 16)) if name.startswith("2d") else fi.cantilever_3d((8, 4, 4))
    m = w.mesh
    print("case alloc %s" % name, flush=True)
    ctx = fo.Context.from_workload(w)
    n, N = m.n_dofs, m.n_nodes
    z = lambda k, dt=torch.float64: torch.zeros(k, dtype=dt, device="cuda")
    phi, b = dev(w.phi), dev(w.b.reshape(-1))
    u, rhs, theta, J, vol, btt = z(n), z(n), z(n), z(1), z(1), z(1)
    hb, hu, hr = z(N), z(N), z(n)
    f = dev(np.ones(N))
    g0 = dev((np.abs(m.coords[:, 0]) < 1e-12).astype(np.uint8), np.uint8)
    dopts = fo.DescentOpts(w.alpha, w.gamma_n, w.gamma_s, w.boxes, dim=m.dim)
    torch.cuda.synchronize()
    before = fo.device_allocations()
    for prec in (fo.FO_FP64, fo.FO_FP32_IR):
        ctx.set_levelset(phi)
        ctx.state_solve(b, u, fo.SolveOpts(precision=prec, rtol=1e-10))
        ctx.shape_derivative(u, rhs, J, vol, lambda_vol=0.3, V=1.0)
        ctx.descent_solve(dopts, rhs, theta, fo.SolveOpts(precision=prec, rtol=1e-10), B_tt=btt)
        ctx.levelset_update(theta, 1e-3, phi)
        ctx.transport(theta, 1e-3, 2, phi)
        ctx.reinit(phi, steps=2, t_end=0.01)
        ctx.heat_load(f, hb)
        ctx.heat_solve(g0, hb, hu, fo.SolveOpts(rtol=1e-10))
        ctx.heat_derivative(hu, f, hr, J, vol)
    torch.cuda.synchronize()
    assert fo.device_allocations() == before
    assert np.isfinite(phi.cpu().numpy()).all()
    ctx.close()
