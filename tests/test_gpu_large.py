"""The large single instances: one full iteration (state, derivative,
velocity, update) on 64x32x32 cubes x 6 tetrahedra against the oracle's
iteration, in FP64 and in FP32 + refinement (its error is measured on this
mesh, where the oracle runs to 1e-12), and on the paper's 3D mesh size
120x60x60 cubes x 6 tetrahedra (2.59M elements) and on 256x128x128 (25.2M
elements, 12.8M unknowns) in the configuration bench.py times, checked on
sampled nodes: the oracle assembles the elements around each sampled node,
which gives that node's rows of K u, of the velocity operator and of the
derivative exactly, and its updated level set."""
import numpy as np
import pytest

import fo_inputs as fi
import oracle as oc

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from paper_2601_05709_amd import fo  # noqa: E402
from paper_2601_05709_amd.pipeline import Iteration  # noqa: E402


def rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


@pytest.mark.parametrize("precision", [fo.FO_FP64, fo.FO_FP32_IR])
def test_iteration_64x32x32_matches_oracle(precision):
    w = fi.cantilever_3d((64, 32, 32))
    print("case 64x32x32 iteration, precision %d" % precision, flush=True)
    it = Iteration(w, fo.SolveOpts(precision=precision, rtol=1e-11), fo.SolveOpts(precision=precision, rtol=1e-11))
    out = it.run(update=True, lambda_vol=0.2, V=1.5)
    torch.cuda.synchronize()
    ref = oc.run_iteration(w, rtol=1e-12, lambda_vol=0.2, V=1.5, dt=out.dt)
    e_u = rel(out.u[:, 0].cpu().numpy(), ref.u)
    e_rhs = rel(out.rhs.cpu().numpy(), ref.rhs)
    e_J = abs(float(out.J[0]) - ref.J[0]) / abs(ref.J[0])
    e_th = rel(out.theta.cpu().numpy(), ref.theta)
    e_phi = np.abs(it.phi.cpu().numpy() - ref.phi_new).max() / np.abs(ref.phi_new).max()
    print("  u %.2e rhs %.2e J %.2e theta %.2e phi %.2e" % (e_u, e_rhs, e_J, e_th, e_phi), flush=True)
    assert e_u <= 1e-8 and e_rhs <= 1e-6 and e_J <= 1e-6
    assert e_th <= 1e-6 and e_phi <= 1e-10
    # the oracle adds the 393,216 element volumes in a plain loop: its rounding
    # bound is about n eps = 4.4e-11 relative
    assert float(out.vol) == pytest.approx(ref.vol, rel=1e-10)


def patch(m, nodes):
    """Elements and boundary facets with a vertex among `nodes`."""
    mark = np.zeros(m.n_nodes, dtype=bool)
    mark[nodes] = True
    conn = np.ascontiguousarray(m.conn[:, mark[m.conn].any(axis=0)])
    fsel = mark[m.bfacets].any(axis=0)
    return conn, np.ascontiguousarray(m.bfacets[:, fsel]), np.ascontiguousarray(m.bnormal[fsel])


@pytest.mark.parametrize("cells", [(120, 60, 60), (256, 128, 128)], ids=["120x60x60", "256x128x128"])
def test_iteration_large_on_sampled_nodes(cells):
    w = fi.cantilever_3d(cells)
    m = w.mesh
    d = m.dim
    tag = "x".join(map(str, cells))
    print("case %s: context (%d elements, %d unknowns)" % (tag, m.n_elems, m.n_dofs), flush=True)
    it = Iteration(w, fo.SolveOpts(precision=fo.FO_FP32_IR, rtol=1e-8),
                   fo.SolveOpts(precision=fo.FO_FP32_IR, rtol=1e-8))
    ts = it.ctx.tile_stats()
    assert ts["n_tiles"] > 0 and ts["n_slots"] >= m.n_nodes
    print("case %s: iteration" % tag, flush=True)
    out = it.run(update=True)
    torch.cuda.synchronize()
    assert out.state_stats.status == 0 and out.state_stats.rel_res <= 1e-8
    assert out.descent_stats.status == 0 and out.descent_stats.rel_res <= 1e-8
    u = out.u[:, 0].cpu().numpy()
    rhs, theta, phi = out.rhs.cpu().numpy(), out.theta.cpu().numpy(), it.phi.cpu().numpy()
    b = w.b.reshape(-1)
    bn = np.linalg.norm(b)
    # cost: b . u equals the energy sum to the solve's tolerance
    assert float(out.J[0]) == pytest.approx(float(b @ u), rel=1e-6)
    lam, mu = oc.lame(w.E, w.nu, d, w.plane_stress)
    A_all, chi_all = oc.element_coef(d, m.conn, w.phi, w.ersatz)
    vol_ref = float(np.sum(chi_all * np.abs(np.linalg.det(
        np.stack([m.coords[m.conn[a]] - m.coords[m.conn[0]] for a in range(1, d + 1)], axis=1))) / 6.0))
    assert float(out.vol) == pytest.approx(vol_ref, rel=1e-9)
    rng = np.random.default_rng(8)
    nodes = np.unique(np.concatenate([rng.integers(0, m.n_nodes, 1500),
                                      np.flatnonzero(np.abs(m.coords[:, 0] - 2.0) < 1e-12)[::97]]))
    conn, bf, bnorm = patch(m, nodes)
    A_e, chi = oc.element_coef(d, conn, w.phi, w.ersatz)
    rows = (nodes[:, None] * d + np.arange(d)).ravel()
    free = w.fixed[rows] == 0
    # state: the sampled rows of the residual b - K u
    K = oc.assemble_elasticity(d, m.coords, conn, A_e, lam, mu)
    r = (b - K.matvec(u))[rows][free]
    print("case %s: max sampled state residual %.2e of ||b||" % (tag, np.abs(r).max() / bn), flush=True)
    assert np.abs(r).max() <= 1e-8 * bn
    assert np.all(u[rows][~free] == 0.0)
    # derivative: the sampled rows, recomputed by the oracle from the same u
    rhs_ref, _, _, _ = oc.shape_derivative(d, m.coords, conn, A_e, chi, lam, mu, u)
    assert np.abs(rhs[rows] - rhs_ref[rows]).max() <= 1e-12 * np.abs(rhs_ref[rows]).max()
    # velocity: the sampled rows of the residual rhs - B theta
    Bd = oc.assemble_descent(d, m.coords, conn, bf, bnorm, w.alpha, w.gamma_n, w.gamma_s, w.boxes)
    rd = (rhs - Bd.matvec(theta))[rows]
    assert np.abs(rd).max() <= 1e-8 * np.linalg.norm(rhs)
    # update: the sampled nodes' new level set
    ref = oc.levelset_update(d, m.coords, conn, theta, out.dt, w.phi)
    assert np.abs(phi[nodes] - ref[nodes]).max() <= 1e-13 * np.abs(w.phi).max()
