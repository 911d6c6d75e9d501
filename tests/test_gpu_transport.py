"""GPU parity of the paper's transport step (fo_transport: Crank-Nicolson
Petrov-Galerkin with optional h^2 diffusion, Jacobi BiCGStab in FP64)
against the FP64 oracle, through the C ABI."""
import numpy as np
import pytest

import fo_inputs as fi
import oracle as oc

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from paper_2601_05709_amd import fo  # noqa: E402

WORKLOADS = {
    "2d_37x19": lambda: fi.cantilever_2d((37, 19)),
    "3d_12x6x6": lambda: fi.cantilever_3d((12, 6, 6)),
    "3d_26x13x11": lambda: fi.cantilever_3d((26, 13, 11)),
}


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).cuda()


def smooth_velocity(coords, seed):
    """A smooth synthetic velocity field of the size a descent solve gives."""
    rng = np.random.default_rng(seed)
    d = coords.shape[1]
    k = rng.uniform(1.0, 3.0, size=(d, d))
    ph = rng.uniform(0, 2 * np.pi, size=d)
    th = np.stack([np.sin(coords @ k[i] + ph[i]) for i in range(d)], axis=1)
    return 0.8 * th


@pytest.mark.parametrize("name", list(WORKLOADS))
@pytest.mark.parametrize("smooth", [True, False])
def test_transport_matches_oracle(name, smooth):
    w = WORKLOADS[name]()
    m = w.mesh
    theta = smooth_velocity(m.coords, 21).ravel()
    dt, steps = 0.006, 5
    ref, _ = oc.transport(m.dim, m.coords, m.conn, theta, dt, steps, w.phi, smooth=smooth, rtol=1e-13)
    ctx = fo.Context.from_workload(w)
    phi = dev(w.phi)
    st = ctx.transport(dev(theta), dt, steps, phi, fo.SolveOpts(rtol=1e-12), smooth=smooth)
    assert st.status == 0 and st.iters_outer == steps and st.iters_inner > 0
    assert st.rel_res <= 1e-12
    got = phi.cpu().numpy()
    assert np.linalg.norm(got - ref) <= 1e-10 * np.linalg.norm(ref)
    # the step moved phi
    assert np.linalg.norm(ref - w.phi) > 1e-4 * np.linalg.norm(w.phi)


@pytest.mark.parametrize("name", ["2d_37x19", "3d_12x6x6"])
def test_transport_moves_a_linear_field_exactly(name):
    """Constant velocity, no diffusion: a linear phi is transported exactly."""
    w = WORKLOADS[name]()
    m = w.mesh
    a = np.array([0.7, -0.4, 0.3][:m.dim])
    th = np.array([0.25, 0.1, -0.2][:m.dim])
    phi0 = m.coords @ a + 0.3
    ctx = fo.Context.from_workload(w)
    phi = dev(phi0)
    ctx.transport(dev(np.tile(th, m.n_nodes)), 0.02, 4, phi, fo.SolveOpts(rtol=1e-13), smooth=False)
    np.testing.assert_allclose(phi.cpu().numpy(), phi0 - 4 * 0.02 * (a @ th), rtol=0, atol=1e-11)


def test_transport_edge_cases():
    w = WORKLOADS["2d_37x19"]()
    m = w.mesh
    ctx = fo.Context.from_workload(w)
    phi = dev(w.phi)
    # zero steps: unchanged
    st = ctx.transport(dev(np.zeros(m.n_dofs)), 0.01, 0, phi)
    assert st.iters_outer == 0
    assert torch.equal(phi, dev(w.phi))
    # no velocity and no diffusion: the step is the identity
    ctx.transport(dev(np.zeros(m.n_dofs)), 0.05, 3, phi, fo.SolveOpts(rtol=1e-13), smooth=False)
    np.testing.assert_allclose(phi.cpu().numpy(), w.phi, rtol=0, atol=1e-12)
    # a constant stays constant under diffusion and any velocity
    c = dev(np.full(m.n_nodes, 1.5))
    ctx.transport(dev(smooth_velocity(m.coords, 3).ravel()), 0.01, 2, c, fo.SolveOpts(rtol=1e-13))
    np.testing.assert_allclose(c.cpu().numpy(), 1.5, rtol=0, atol=1e-11)
    # invalid arguments are refused before anything runs
    with pytest.raises(fo.FoError):
        ctx.transport(dev(np.zeros(m.n_dofs)), -0.01, 1, phi)
    with pytest.raises(fo.FoError):
        ctx.transport(dev(np.zeros(m.n_dofs)), 0.01, -1, phi)
    # the atomic scatter has no transport operator
    ctx.set_scatter(fo.FO_SCATTER_ATOMIC)
    with pytest.raises(fo.FoError):
        ctx.transport(dev(np.zeros(m.n_dofs)), 0.01, 1, phi)


def test_transport_after_a_descent_solve_matches_oracle():
    """The hot-path sequence: descent velocity, then the paper's transport
    with its adaptive final time and step count."""
    w = WORKLOADS["3d_12x6x6"]()
    m = w.mesh
    rng = np.random.default_rng(5)
    rhs = rng.standard_normal(m.n_dofs)
    Bd = oc.assemble_descent(m.dim, m.coords, m.conn, m.bfacets, m.bnormal, w.alpha, w.gamma_n,
                             w.gamma_s, w.boxes)
    theta, _ = Bd.solve(rhs, None, rtol=1e-12)
    t_end, steps, dt = oc.adaptive_dt(float(theta @ rhs))
    ref, _ = oc.transport(m.dim, m.coords, m.conn, theta, dt, steps, w.phi, smooth=True, rtol=1e-13)
    ctx = fo.Context.from_workload(w)
    phi = dev(w.phi)
    st = ctx.transport(dev(theta), dt, steps, phi, fo.SolveOpts(rtol=1e-12))
    assert st.status == 0 and st.iters_outer == steps
    assert np.linalg.norm(phi.cpu().numpy() - ref) <= 1e-10 * np.linalg.norm(ref)


def test_repeated_calls_reuse_the_captured_solver():
    """The solver's iterations are captured once per context and replayed:
    later calls with another dt, another velocity array (at another address)
    and the diffusion switched off still match the oracle."""
    w = WORKLOADS["3d_12x6x6"]()
    m = w.mesh
    ctx = fo.Context.from_workload(w)
    cases = [(0.006, 4, 21, True), (0.011, 3, 22, False), (0.003, 5, 23, True)]
    for dt, steps, seed, smooth in cases:
        theta = smooth_velocity(m.coords, seed).ravel()
        ref, _ = oc.transport(m.dim, m.coords, m.conn, theta, dt, steps, w.phi, smooth=smooth, rtol=1e-13)
        th_dev = dev(theta)  # a fresh allocation each call
        phi = dev(w.phi)
        print("case transport dt %g steps %d seed %d smooth %s" % (dt, steps, seed, smooth), flush=True)
        st = ctx.transport(th_dev, dt, steps, phi, fo.SolveOpts(rtol=1e-12), smooth=smooth)
        assert st.status == 0 and st.iters_outer == steps
        assert np.linalg.norm(phi.cpu().numpy() - ref) <= 1e-10 * np.linalg.norm(ref)


def test_iteration_limit_reports_not_converged():
    """A cap on operator applications below what a step needs ends the call
    with FO_NOT_CONVERGED (raised unless allowed) and leaves phi finite."""
    w = WORKLOADS["3d_12x6x6"]()
    m = w.mesh
    ctx = fo.Context.from_workload(w)
    theta = dev(smooth_velocity(m.coords, 9).ravel())
    phi = dev(w.phi)
    with pytest.raises(fo.FoError):
        ctx.transport(theta, 0.01, 2, phi, fo.SolveOpts(rtol=1e-14, max_iter=2))
    phi = dev(w.phi)
    st = ctx.transport(theta, 0.01, 2, phi, fo.SolveOpts(rtol=1e-14, max_iter=2), allow_not_converged=True)
    assert st.status == fo.FO_NOT_CONVERGED
    assert torch.isfinite(phi).all()
    # the same context still solves to tolerance afterwards
    ref, _ = oc.transport(m.dim, m.coords, m.conn, theta.cpu().numpy(), 0.01, 2, w.phi, smooth=True, rtol=1e-13)
    phi = dev(w.phi)
    st = ctx.transport(theta, 0.01, 2, phi, fo.SolveOpts(rtol=1e-12))
    assert st.status == 0
    assert np.linalg.norm(phi.cpu().numpy() - ref) <= 1e-10 * np.linalg.norm(ref)
