"""Seeded input generators: mesh structure, loads, masks, level sets."""
import numpy as np
import pytest

import fo_inputs as fi


def signed_measures(m):
    X, Cn = m.coords, m.conn
    a = X[Cn[1]] - X[Cn[0]]
    b = X[Cn[2]] - X[Cn[0]]
    if m.dim == 2:
        return 0.5 * (a[:, 0] * b[:, 1] - a[:, 1] * b[:, 0])
    c = X[Cn[3]] - X[Cn[0]]
    return np.einsum("ij,ij->i", a, np.cross(b, c)) / 6.0


def facets_of(m):
    """All facets (sorted node tuples) with their multiplicity."""
    Cn = m.conn.T
    faces = np.concatenate([np.delete(Cn, s, axis=1) for s in range(m.dim + 1)])
    return np.unique(np.sort(faces, axis=1), axis=0, return_counts=True)


@pytest.mark.parametrize("cells,lengths", [((4, 3), (2.0, 1.0)), ((64, 32), (2.0, 1.0)),
                                           ((3, 2, 2), (2.0, 1.0, 1.0)), ((6, 3, 3), (2.0, 1.0, 1.0))])
def test_mesh_counts_volumes_conformity(cells, lengths):
    m = fi.structured_mesh(cells, lengths)
    nn = int(np.prod([c + 1 for c in cells]))
    ne = int(np.prod(cells)) * (2 if len(cells) == 2 else 6)
    assert m.n_nodes == nn and m.n_elems == ne
    v = signed_measures(m)
    assert np.all(np.abs(v) > 0)
    cell = np.prod([L / n for L, n in zip(lengths, cells)])
    np.testing.assert_allclose(np.abs(v), cell / (2 if m.dim == 2 else 6), rtol=1e-12)
    assert abs(np.abs(v).sum() - np.prod(lengths)) < 1e-12 * np.prod(lengths)
    faces, cnt = facets_of(m)
    assert cnt.max() == 2  # every interior facet is shared by exactly two elements
    bnd = faces[cnt == 1]
    ours = np.unique(np.sort(m.bfacets.T, axis=1), axis=0)
    assert np.array_equal(bnd, ours)
    # outward normals: facet nodes lie on the face the normal points out of
    for f in range(m.bfacets.shape[1]):
        ax = int(np.argmax(np.abs(m.bnormal[f])))
        side = m.bnormal[f, ax]
        assert abs(abs(side) - 1.0) == 0.0
        target = 0.0 if side < 0 else lengths[ax]
        assert np.all(m.coords[m.bfacets[:, f], ax] == target)


def test_config_sizes():
    m = fi.structured_mesh((96, 48, 48), (2.0, 1.0, 1.0))
    assert (m.n_nodes, m.n_elems, m.n_dofs) == (232897, 1327104, 698691)
    m = fi.structured_mesh((64, 32, 32), (2.0, 1.0, 1.0))
    assert (m.n_nodes, m.n_elems) == (70785, 393216)
    m = fi.structured_mesh((64, 32), (2.0, 1.0))
    assert (m.n_nodes, m.n_elems, m.n_dofs) == (2145, 4096, 4290)


def test_load_total_equals_traction_times_patch():
    w = fi.cantilever_2d()
    np.testing.assert_allclose(w.b.reshape(-1, 2).sum(0), [0.0, -0.1], atol=1e-15)
    w3 = fi.cantilever_3d((12, 6, 6))
    np.testing.assert_allclose(w3.b.reshape(-1, 3).sum(0), [0.0, 0.0, -0.01], atol=1e-15)
    # loaded nodes lie on x = 2 only
    nz = np.nonzero(np.abs(w3.b.reshape(-1, 3)).sum(1))[0]
    assert np.all(w3.mesh.coords[nz, 0] == 2.0)


def test_load_matches_fine_quadrature():
    """Clipped exact integration vs brute-force quadrature on a fine lattice of
    sample points (midpoint rule with 400x400 points on the patch)."""
    m = fi.structured_mesh((8, 4, 4), (2.0, 1.0, 1.0))
    lo, hi = (0.31, 0.47), (0.52, 0.61)
    b = fi.traction_load(m, (1.0, 0.0, 0.0), lo, hi)
    n = 400
    ys = lo[0] + (np.arange(n) + 0.5) * (hi[0] - lo[0]) / n
    zs = lo[1] + (np.arange(n) + 0.5) * (hi[1] - lo[1]) / n
    Y, Z = np.meshgrid(ys, zs, indexing="ij")
    Y, Z = Y.ravel(), Z.ravel()
    dA = (hi[0] - lo[0]) * (hi[1] - lo[1]) / n ** 2
    ref = np.zeros(m.n_nodes)
    # hat functions of the face triangulation evaluated at the sample points
    sel = m.bnormal[:, 0] == 1.0
    for f in m.bfacets[:, sel].T:
        P = m.coords[f][:, 1:]
        T = np.array([P[1] - P[0], P[2] - P[0]]).T
        l12 = np.linalg.solve(T, np.stack([Y - P[0, 0], Z - P[0, 1]]))
        l0 = 1 - l12[0] - l12[1]
        inside = (l0 >= -1e-14) & (l12[0] >= -1e-14) & (l12[1] >= -1e-14)
        # points on shared edges belong to one facet only
        owned = inside & ~np.isnan(Y)
        for node, lam in zip(f, (l0, l12[0], l12[1])):
            ref[node] += np.where(owned, lam, 0.0).sum() * dA
        Y = np.where(owned, np.nan, Y)
    got = b.reshape(-1, 3)[:, 0]
    np.testing.assert_allclose(got.sum(), 0.21 * 0.14, rtol=1e-12)
    assert np.max(np.abs(got - ref)) < 2e-5 * np.max(np.abs(ref))


def test_clamp_and_levelsets():
    w = fi.cantilever_3d((8, 4, 4))
    fixed_nodes = np.nonzero(w.fixed.reshape(-1, 3).all(1))[0]
    assert np.all(w.mesh.coords[fixed_nodes, 0] == 0.0)
    assert len(fixed_nodes) == 5 * 5
    c = fi.sphere_hole_centers_4x2x2()
    assert c.shape == (16, 3)
    phi = fi.levelset_balls(c, c, 0.15)
    np.testing.assert_allclose(phi, 0.15)  # at the centres: inside a hole (phi > 0)
    phi_u = fi.levelset_balls(c, c, 0.15, factor=-1.0)
    np.testing.assert_allclose(phi_u, -0.15)
    x = np.array([[0.0, 0.0], [0.125, 0.0]])
    np.testing.assert_allclose(fi.levelset_cos_holes(x), [-1.4, -0.4 - np.cos(np.pi / 2)],
                               atol=1e-15)


def test_seeded_generators_are_deterministic():
    a = fi.multi_load_3d((8, 4, 4), n_loads=5)
    b = fi.multi_load_3d((8, 4, 4), n_loads=5)
    assert np.array_equal(a.b, b.b)
    np.testing.assert_allclose(np.abs(a.b.reshape(-1, 3, 5).sum(0)).sum(0) > 0, True)
    r1 = fi.serving_request(7)
    r2 = fi.serving_request(7)
    assert r1.name == r2.name and np.array_equal(r1.phi, r2.phi) and np.array_equal(r1.b, r2.b)
    t = fi.poisson_arrivals(1000)
    assert np.all(np.diff(t) > 0) and 3.0 < t[-1] < 7.0


def test_inverse_pairs():
    """Pair 0 of a multi-pair inverse workload is the single-pair workload;
    every pair's traction integrates to its direction times the patch
    measure, and every g_k vanishes on Gamma_0."""
    for cells, area in (((24, 12), 0.4), ((8, 4, 4), 0.16)):
        one = fi.inverse_elasticity(cells)
        w = fi.inverse_elasticity(cells, n_pairs=4)
        d = len(cells)
        assert w.n_pairs == 4 and one.n_pairs == 1
        assert np.array_equal(w.fs[0], one.f) and np.array_equal(w.gs[0], one.g)
        for k in range(4):
            t = w.fs[k].reshape(-1, d).sum(axis=0)
            ang = 0.35 * k
            expect = np.array((-np.cos(ang), np.sin(ang)) + ((0.5 * np.sin(ang),) if d == 3 else ())) * area
            np.testing.assert_allclose(t, expect, atol=1e-12)
            assert np.all(w.gs[k][w.fixed0 == 1] == 0.0)
            pk = w.pair(k)
            assert pk.n_pairs == 1 and pk.f is w.fs[k] and pk.g is w.gs[k]
        assert w.columns(w.fs).shape == (w.mesh.n_dofs, 4)
