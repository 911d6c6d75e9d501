"""Host-side pieces of the serving path (no GPU): footprint estimate from the
mesh sizes alone, latency percentiles, pool creation failing cleanly without
a device, and the mesh-identity key used for context reuse."""
import ctypes as C

import numpy as np
import pytest

import fo_inputs as fi
from paper_2601_05709_amd import fo, serving


def estimate(w):
    m = w.mesh
    coords = np.ascontiguousarray(m.coords)
    conn = np.ascontiguousarray(m.conn, dtype=np.int32)
    bf = np.ascontiguousarray(m.bfacets, dtype=np.int32)
    bn = np.ascontiguousarray(m.bnormal)
    mesh = fo.fo_mesh(m.dim, m.n_nodes, m.n_elems, coords.ctypes.data, conn.ctypes.data, None,
                      int(bf.shape[1]), bf.ctypes.data, bn.ctypes.data)
    return fo.lib().fo_footprint_estimate(C.byref(mesh))


def test_footprint_estimate_grows_with_the_mesh_and_covers_the_vectors():
    sizes = [fi.cantilever_2d((32, 16)), fi.cantilever_2d((64, 32)), fi.cantilever_3d((8, 4, 4), holes=False),
             fi.cantilever_3d((16, 8, 8), holes=False)]
    est = [estimate(w) for w in sizes]
    assert est[0] < est[1] and est[2] < est[3]
    for w, e in zip(sizes, est):
        n = w.mesh.n_dofs
        assert e > n * (8 * 9 + 4 * 7)  # at least the Krylov and diagonal vectors


def test_footprint_estimate_rejects_invalid_mesh():
    mesh = fo.fo_mesh(4, 10, 10, None, None, None, 0, None, None)
    assert fo.lib().fo_footprint_estimate(C.byref(mesh)) == 0
    mesh = fo.fo_mesh(3, 0, 10, None, None, None, 0, None, None)
    assert fo.lib().fo_footprint_estimate(C.byref(mesh)) == 0


def test_percentile_matches_numpy_linear():
    rng = np.random.default_rng(0)
    x = rng.exponential(size=137)
    for q in (0, 1, 50, 90, 99, 100):
        assert serving.percentile(x, q) == pytest.approx(np.percentile(x, q), rel=1e-12)


def test_mesh_key_identifies_mesh_and_material():
    a = fi.serving_request(0, meshes=(("2d", (16, 8)),))
    b = fi.serving_request(1, meshes=(("2d", (16, 8)),))
    c = fi.serving_request(2, meshes=(("2d", (24, 8)),))
    assert serving.mesh_key(a) == serving.mesh_key(b) != 0
    assert serving.mesh_key(a) != serving.mesh_key(c)
    assert not np.array_equal(a.phi, b.phi)  # same mesh, different level sets


def test_pool_arguments_are_checked_on_the_host():
    h = C.c_void_p()
    assert fo.lib().fo_pool_create(C.byref(h), 0, 4) == fo.FO_ERR_ARG
    assert fo.lib().fo_pool_create(C.byref(h), 1 << 20, 0) == fo.FO_ERR_ARG
    assert fo.lib().fo_pool_create(C.byref(h), 1 << 20, 65) == fo.FO_ERR_ARG
    assert fo.lib().fo_pool_admit(None, None, None) == fo.FO_ERR_ARG
    assert fo.lib().fo_pool_release(None, 0) == fo.FO_ERR_ARG
    assert fo.lib().fo_status_string(fo.FO_ERR_BUSY).decode().startswith("no free slot")
