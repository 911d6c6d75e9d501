"""Parity of the HIP path (through the C ABI) with the FP64 CPU oracle.

Tolerances: operator applications and element passes agree to rounding
(1e-13 relative in FP64, 1e-5 in FP32 geometry); solves agree to the
spec bars (displacement 1e-8, shape derivative and J 1e-6) and in
practice much tighter because both sides solve to small residuals.
"""
import numpy as np
import pytest

import fo_inputs as fi
import oracle as oc

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from paper_2601_05709_amd import fo  # noqa: E402
from paper_2601_05709_amd.pipeline import Iteration  # noqa: E402


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def rel(a, b):
    return np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300)


def relmax(a, b):
    return np.abs(a - b).max() / max(np.abs(b).max(), 1e-300)


WORKLOADS = {
    "2d_64x32": lambda: fi.cantilever_2d((64, 32)),
    "2d_37x19": lambda: fi.cantilever_2d((37, 19)),
    "3d_12x6x6": lambda: fi.cantilever_3d((12, 6, 6)),
    "3d_26x13x11": lambda: fi.cantilever_3d((26, 13, 11)),
}


def oracle_K(w):
    m = w.mesh
    lam, mu = oc.lame(w.E, w.nu, m.dim, w.plane_stress)
    A, chi = oc.element_coef(m.dim, m.conn, w.phi, w.ersatz)
    return oc.assemble_elasticity(m.dim, m.coords, m.conn, A, lam, mu), A, chi, lam, mu


@pytest.mark.parametrize("name", list(WORKLOADS))
@pytest.mark.parametrize("scatter", [fo.FO_SCATTER_TILED, fo.FO_SCATTER_ATOMIC])
def test_elasticity_apply_fp64(name, scatter):
    w = WORKLOADS[name]()
    print("case", name, scatter, flush=True)
    K, *_ = oracle_K(w)
    ctx = fo.Context.from_workload(w)
    ctx.set_scatter(scatter)
    ctx.set_levelset(dev(w.phi))
    x = np.random.default_rng(1).standard_normal(w.mesh.n_dofs)
    x[w.fixed == 1] = 0.0
    y = torch.zeros(w.mesh.n_dofs, dtype=torch.float64, device="cuda")
    ctx.apply_elasticity(dev(x), y)
    ref = K.matvec(x)
    ref[w.fixed == 1] = 0.0
    assert relmax(y.cpu().numpy(), ref) < 1e-13


@pytest.mark.parametrize("name", ["2d_64x32", "3d_26x13x11"])
def test_elasticity_apply_fp32(name):
    w = WORKLOADS[name]()
    K, *_ = oracle_K(w)
    ctx = fo.Context.from_workload(w)
    ctx.set_levelset(dev(w.phi))
    x = np.random.default_rng(2).standard_normal(w.mesh.n_dofs)
    x[w.fixed == 1] = 0.0
    y = torch.zeros(w.mesh.n_dofs, dtype=torch.float32, device="cuda")
    ctx.apply_elasticity(dev(x.astype(np.float32)), y, precision=fo.FO_FP32_IR)
    ref = K.matvec(x)
    ref[w.fixed == 1] = 0.0
    assert relmax(y.double().cpu().numpy(), ref) < 1e-5


def test_tiled_apply_is_bitwise_reproducible():
    w = WORKLOADS["3d_26x13x11"]()
    ctx = fo.Context.from_workload(w)
    ctx.set_levelset(dev(w.phi))
    x = dev(np.random.default_rng(3).standard_normal(w.mesh.n_dofs))
    ys = []
    for _ in range(3):
        y = torch.empty(w.mesh.n_dofs, dtype=torch.float64, device="cuda")
        ctx.apply_elasticity(x, y)
        ys.append(y.cpu().numpy())
    assert np.array_equal(ys[0], ys[1]) and np.array_equal(ys[0], ys[2])


@pytest.mark.parametrize("name", ["2d_64x32", "3d_12x6x6"])
@pytest.mark.parametrize("precision", [fo.FO_FP64, fo.FO_FP32_IR])
def test_state_solve(name, precision):
    w = WORKLOADS[name]()
    print("case", name, precision, flush=True)
    K, *_ = oracle_K(w)
    u_ref, info = K.solve(w.b, w.fixed, rtol=1e-12)
    ctx = fo.Context.from_workload(w)
    ctx.set_levelset(dev(w.phi))
    u = torch.zeros(w.mesh.n_dofs, dtype=torch.float64, device="cuda")
    st = ctx.state_solve(dev(w.b), u, fo.SolveOpts(precision=precision, rtol=1e-11))
    uh = u.cpu().numpy()
    assert st.status == 0 and st.rel_res <= 1e-11
    assert rel(uh, u_ref) < 1e-8
    # the oracle's residual of the GPU solution
    r = w.b - K.matvec(uh)
    r[w.fixed == 1] = 0.0
    bf = w.b.copy()
    bf[w.fixed == 1] = 0.0
    assert np.linalg.norm(r) <= 2e-11 * np.linalg.norm(bf)
    assert np.all(uh[w.fixed == 1] == 0.0)
    if precision == fo.FO_FP32_IR:
        assert st.iters_outer >= 1


@pytest.mark.parametrize("name", ["2d_37x19", "3d_26x13x11"])
@pytest.mark.parametrize("scatter", [fo.FO_SCATTER_TILED, fo.FO_SCATTER_ATOMIC])
def test_shape_derivative_matches_oracle(name, scatter):
    w = WORKLOADS[name]()
    m = w.mesh
    K, A, chi, lam, mu = oracle_K(w)
    n_rhs, ld = 3, 4
    rng = np.random.default_rng(4)
    U = rng.standard_normal((m.n_dofs, ld))
    rhs_ref, S1_ref, J_ref, vol_ref = oc.shape_derivative(m.dim, m.coords, m.conn, A, chi, lam, mu,
                                                          U[:, :n_rhs], lambda_vol=0.7, V=1.3,
                                                          want_S1=True)
    ctx = fo.Context.from_workload(w, max_rhs=4)
    ctx.set_scatter(scatter)
    ctx.set_levelset(dev(w.phi))
    rhs = torch.zeros(m.n_dofs, dtype=torch.float64, device="cuda")
    S1 = torch.zeros(m.dim * m.dim * m.n_elems, dtype=torch.float64, device="cuda")
    J = torch.zeros(n_rhs, dtype=torch.float64, device="cuda")
    vol = torch.zeros(1, dtype=torch.float64, device="cuda")
    ctx.shape_derivative(dev(U), rhs, J, vol, n_rhs=n_rhs, ld=ld, lambda_vol=0.7, V=1.3, S1=S1)
    assert relmax(rhs.cpu().numpy(), rhs_ref) < 1e-12
    assert relmax(S1.cpu().numpy(), S1_ref.ravel()) < 1e-12
    np.testing.assert_allclose(J.cpu().numpy(), J_ref, rtol=1e-12)
    assert vol.item() == pytest.approx(vol_ref, rel=1e-13)


@pytest.mark.parametrize("name", ["2d_37x19", "3d_12x6x6"])
def test_descent_apply_and_solve(name):
    w = WORKLOADS[name]()
    m = w.mesh
    Bd = oc.assemble_descent(m.dim, m.coords, m.conn, m.bfacets, m.bnormal, w.alpha, w.gamma_n,
                             w.gamma_s, w.boxes)
    ctx = fo.Context.from_workload(w)
    dop = fo.DescentOpts(w.alpha, w.gamma_n, w.gamma_s, w.boxes, dim=m.dim)
    x = np.random.default_rng(5).standard_normal(m.n_dofs)
    y = torch.zeros(m.n_dofs, dtype=torch.float64, device="cuda")
    ctx.apply_descent(dop, dev(x), y)
    assert relmax(y.cpu().numpy(), Bd.matvec(x)) < 1e-13
    rhs = np.random.default_rng(6).standard_normal(m.n_dofs)
    th_ref, _ = Bd.solve(rhs, None, rtol=1e-12)
    th = torch.zeros(m.n_dofs, dtype=torch.float64, device="cuda")
    Btt = torch.zeros(1, dtype=torch.float64, device="cuda")
    st = ctx.descent_solve(dop, dev(rhs), th, fo.SolveOpts(rtol=1e-11), Btt)
    assert st.status == 0
    assert rel(th.cpu().numpy(), th_ref) < 1e-8
    assert Btt.item() == pytest.approx(th_ref @ rhs, rel=1e-9)


@pytest.mark.parametrize("name", ["2d_37x19", "3d_12x6x6", "3d_26x13x11"])
def test_descent_solve_fp32_ir(name):
    """FP32 fused descent CG with FP64 residual replacement reaches the same
    FP64 tolerance as the FP64 solve (facet term in the tile kernel)."""
    w = WORKLOADS[name]()
    m = w.mesh
    Bd = oc.assemble_descent(m.dim, m.coords, m.conn, m.bfacets, m.bnormal, w.alpha, w.gamma_n,
                             w.gamma_s, w.boxes)
    ctx = fo.Context.from_workload(w)
    dop = fo.DescentOpts(w.alpha, w.gamma_n, w.gamma_s, w.boxes, dim=m.dim)
    rhs = np.random.default_rng(16).standard_normal(m.n_dofs)
    th_ref, _ = Bd.solve(rhs, None, rtol=1e-12)
    th = torch.zeros(m.n_dofs, dtype=torch.float64, device="cuda")
    Btt = torch.zeros(1, dtype=torch.float64, device="cuda")
    st = ctx.descent_solve(dop, dev(rhs), th, fo.SolveOpts(precision=fo.FO_FP32_IR, rtol=1e-10), Btt)
    assert st.status == 0 and st.iters_outer >= 1
    r = rhs - Bd.matvec(th.cpu().numpy())
    assert np.linalg.norm(r) <= 1.05e-10 * np.linalg.norm(rhs)
    assert rel(th.cpu().numpy(), th_ref) < 1e-7
    assert Btt.item() == pytest.approx(th_ref @ rhs, rel=1e-8)


@pytest.mark.parametrize("name", ["2d_37x19", "3d_12x6x6"])
def test_descent_fused_matches_node_parallel_facets(name):
    """The fused descent CG (facets per tile node) and the generic CG on the
    atomic scatter (node-parallel facets) solve the same system."""
    w = WORKLOADS[name]()
    m = w.mesh
    dop = fo.DescentOpts(w.alpha, w.gamma_n, w.gamma_s, w.boxes, dim=m.dim)
    rhs = dev(np.random.default_rng(17).standard_normal(m.n_dofs))
    out = []
    for scatter in (fo.FO_SCATTER_TILED, fo.FO_SCATTER_ATOMIC):
        ctx = fo.Context.from_workload(w)
        ctx.set_scatter(scatter)
        th = torch.zeros(m.n_dofs, dtype=torch.float64, device="cuda")
        st = ctx.descent_solve(dop, rhs, th, fo.SolveOpts(rtol=1e-12))
        assert st.status == 0
        out.append(th.cpu().numpy())
    assert rel(out[0], out[1]) < 1e-9


@pytest.mark.parametrize("name", ["2d_37x19", "3d_26x13x11"])
def test_levelset_update_matches_oracle(name):
    w = WORKLOADS[name]()
    m = w.mesh
    theta = np.random.default_rng(7).standard_normal(m.n_dofs)
    ref = oc.levelset_update(m.dim, m.coords, m.conn, theta, 0.013, w.phi)
    ctx = fo.Context.from_workload(w)
    phi = dev(w.phi.copy())
    ctx.levelset_update(dev(theta), 0.013, phi)
    assert relmax(phi.cpu().numpy(), ref) < 1e-13


@pytest.mark.parametrize("name", ["2d_64x32", "3d_12x6x6"])
@pytest.mark.parametrize("precision", [fo.FO_FP64, fo.FO_FP32_IR])
def test_full_iteration_matches_oracle(name, precision):
    w = WORKLOADS[name]()
    it = Iteration(w, fo.SolveOpts(precision=precision, rtol=1e-11), fo.SolveOpts(rtol=1e-11))
    out = it.run(lambda_vol=0.2, V=1.0, update=True)
    ref = oc.run_iteration(w, rtol=1e-12, lambda_vol=0.2, V=1.0, dt=out.dt)
    assert rel(out.u[:, 0].cpu().numpy(), ref.u) < 1e-8
    assert rel(out.rhs.cpu().numpy(), ref.rhs) < 1e-6
    assert abs(out.J.item() - ref.J[0]) <= 1e-6 * abs(ref.J[0])
    assert out.vol.item() == pytest.approx(ref.vol, rel=1e-13)
    assert rel(out.theta.cpu().numpy(), ref.theta) < 1e-6
    assert out.B_tt.item() == pytest.approx(ref.B_tt, rel=1e-6)
    assert relmax(it.phi.cpu().numpy(), ref.phi_new) < 1e-8


# ------------------------------------------------------------------ edge cases


def test_single_element_meshes():
    for dim in (2, 3):
        P = np.array([[0, 0], [1, 0], [0, 1]], float) if dim == 2 else \
            np.array([[0, 0, 0], [1, 0, 0], [0, 1, 0], [0, 0, 1]], float)
        conn = np.arange(dim + 1, dtype=np.int32).reshape(-1, 1)
        fixed = np.zeros((dim + 1) * dim, np.uint8)
        fixed[:dim * dim] = 1  # clamp all but the last vertex
        b = np.zeros((dim + 1) * dim)
        b[-1] = -1.0
        phi = -np.ones(dim + 1)
        lam, mu = oc.lame(1.0, 0.3, dim, 1 if dim == 2 else 0)
        K = oc.assemble_elasticity(dim, P, conn, np.ones(1), lam, mu)
        u_ref, _ = K.solve(b, fixed, rtol=1e-14)
        ctx = fo.Context(dim, P, conn, fixed, None, None, plane_stress=1 if dim == 2 else 0)
        ctx.set_levelset(dev(phi))
        u = torch.zeros(b.size, dtype=torch.float64, device="cuda")
        st = ctx.state_solve(dev(b), u, fo.SolveOpts(rtol=1e-13))
        assert st.status == 0
        np.testing.assert_allclose(u.cpu().numpy(), u_ref, rtol=1e-10, atol=1e-14)


def test_zero_rhs_and_status_codes():
    w = WORKLOADS["2d_37x19"]()
    ctx = fo.Context.from_workload(w)
    ctx.set_levelset(dev(w.phi))
    u = torch.full((w.mesh.n_dofs,), 5.0, dtype=torch.float64, device="cuda")
    st = ctx.state_solve(torch.zeros(w.mesh.n_dofs, dtype=torch.float64, device="cuda"), u,
                         fo.SolveOpts(rtol=1e-8))
    assert st.status == 0 and float(u.abs().max()) == 0.0
    st = ctx.state_solve(dev(w.b), u, fo.SolveOpts(rtol=1e-12, max_iter=3), allow_not_converged=True)
    assert st.status == fo.FO_NOT_CONVERGED and st.iters_inner <= 4
    bad = w.b.copy()
    bad[np.nonzero(w.fixed == 0)[0][5]] = np.nan
    with pytest.raises(fo.FoError) as e:
        ctx.state_solve(dev(bad), u, fo.SolveOpts(rtol=1e-8))
    assert e.value.status == fo.FO_ERR_BREAKDOWN


def test_state_requires_levelset():
    w = WORKLOADS["2d_37x19"]()
    ctx = fo.Context.from_workload(w)
    u = torch.zeros(w.mesh.n_dofs, dtype=torch.float64, device="cuda")
    with pytest.raises(fo.FoError) as e:
        ctx.state_solve(dev(w.b), u, fo.SolveOpts())
    assert e.value.status == fo.FO_ERR_STATE


# ------------------------------------------------------------------ full size


@pytest.mark.parametrize("precision", [fo.FO_FP64, fo.FO_FP32_IR])
def test_cantilever_96x48x48_residual_checked_by_oracle(precision):
    """Config-size state solve at rel. residual 1e-8: the oracle assembles K
    and measures the residual of the GPU solution; J = b.u vs the element sum."""
    w = fi.cantilever_3d((96, 48, 48))
    print("case 96x48x48", precision, flush=True)
    m = w.mesh
    ctx = fo.Context.from_workload(w)
    ctx.set_levelset(dev(w.phi))
    u = torch.zeros(m.n_dofs, dtype=torch.float64, device="cuda")
    st = ctx.state_solve(dev(w.b), u, fo.SolveOpts(precision=precision, rtol=1e-8))
    assert st.status == 0 and st.rel_res <= 1e-8
    K, *_ = oracle_K(w)
    uh = u.cpu().numpy()
    r = w.b - K.matvec(uh)
    r[w.fixed == 1] = 0.0
    bf = np.where(w.fixed == 1, 0.0, w.b)
    assert np.linalg.norm(r) <= 1.5e-8 * np.linalg.norm(bf)
    J = torch.zeros(1, dtype=torch.float64, device="cuda")
    vol = torch.zeros(1, dtype=torch.float64, device="cuda")
    rhs = torch.zeros(m.n_dofs, dtype=torch.float64, device="cuda")
    ctx.shape_derivative(u, rhs, J, vol)
    assert J.item() == pytest.approx(float(w.b @ uh), rel=1e-6)


def test_ir_finishes_in_fp64_when_fp32_stagnates():
    """2D 256x128 with random holes: Jacobi-PCG needs ~3800 FP64 iterations
    (kappa * eps_32 near 1), so the FP32 phases stagnate; the solve must still
    reach the FP64 residual target (through its FP64 finish) and match the
    oracle."""
    w = fi.serving_request(0)
    assert w.mesh.dim == 2 and w.mesh.cells == (256, 128)
    print("case serving req0 2d 256x128", flush=True)
    m = w.mesh
    ctx = fo.Context.from_workload(w)
    ctx.set_levelset(dev(w.phi))
    u = torch.zeros(m.n_dofs, dtype=torch.float64, device="cuda")
    st = ctx.state_solve(dev(w.b), u, fo.SolveOpts(precision=fo.FO_FP32_IR, rtol=1e-10))
    assert st.status == 0 and st.rel_res <= 1e-10
    assert st.iters_inner < 40000
    K, *_ = oracle_K(w)
    u_ref, _ = K.solve(w.b, w.fixed, rtol=1e-12)
    assert rel(u.cpu().numpy(), u_ref) < 1e-8


@pytest.mark.parametrize("name", ["2d_37x19", "3d_12x6x6"])
def test_element_coef_on_exact_zero_means(name):
    """A_e and chi_e where the vertex mean of phi is exactly 0 (Section 2,
    material where phi < 0, strictly): phi takes small integer values, so every
    vertex sum is exact in either order and both sides decide on the same
    number.  A flipped element changes vol by |T_e| and the apply by a factor
    1/ersatz on its rows, far above the 1e-13 rounding bars."""
    w = WORKLOADS[name]()
    m = w.mesh
    phi = np.random.default_rng(8).integers(-3, 4, size=m.n_nodes).astype(np.float64)
    sums = phi[m.conn].sum(axis=0)
    assert (sums == 0).sum() > m.n_elems // 20, "workload has too few exact-zero means"
    w.phi = phi
    K, A, chi, lam, mu = oracle_K(w)
    assert np.all(chi[sums == 0] == 0.0) and np.all(A[sums == 0] == w.ersatz)
    ctx = fo.Context.from_workload(w, max_rhs=1)
    ctx.set_levelset(dev(phi))
    x = np.random.default_rng(9).standard_normal(m.n_dofs)
    x[w.fixed == 1] = 0.0
    y = torch.zeros(m.n_dofs, dtype=torch.float64, device="cuda")
    ctx.apply_elasticity(dev(x), y)
    ref = K.matvec(x)
    ref[w.fixed == 1] = 0.0
    assert relmax(y.cpu().numpy(), ref) < 1e-13
    U = np.zeros((m.n_dofs, 1))
    rhs = torch.zeros(m.n_dofs, dtype=torch.float64, device="cuda")
    J = torch.zeros(1, dtype=torch.float64, device="cuda")
    vol = torch.zeros(1, dtype=torch.float64, device="cuda")
    ctx.shape_derivative(dev(U), rhs, J, vol, n_rhs=1)
    _, _, _, vol_ref = oc.shape_derivative(m.dim, m.coords, m.conn, A, chi, lam, mu, U)
    assert vol.item() == pytest.approx(vol_ref, rel=1e-13)
