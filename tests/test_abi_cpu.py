"""The C-ABI library loads without a GPU, exports every declared symbol, and
rejects invalid input on the host before touching the device."""
import ctypes as C
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
LIB = os.path.join(ROOT, "paper_2601_05709_amd", "libfo.so")


def declared_symbols():
    names = set()
    inc = os.path.join(ROOT, "include")
    for fn in os.listdir(inc):
        if fn.endswith(".h"):
            text = open(os.path.join(inc, fn)).read()
            text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
            names |= set(re.findall(r"\b(fo_[a-z_0-9]+)\s*\(", text))
    return names


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(LIB):
        from paper_2601_05709_amd import build
        build.build()
    from paper_2601_05709_amd import fo
    return fo.lib()


def test_exports_every_declared_symbol(lib):
    names = declared_symbols()
    assert {"fo_create", "fo_state_solve", "fo_shape_derivative", "fo_descent_solve",
            "fo_levelset_update"} <= names
    for n in sorted(names):
        assert hasattr(lib, n), n


def test_status_strings(lib):
    from paper_2601_05709_amd import fo
    assert fo.status_string(0) == "ok"
    assert "breakdown" in fo.status_string(fo.FO_ERR_BREAKDOWN)


def _create(lib, dim, coords, conn, fixed=None):
    from paper_2601_05709_amd import fo
    coords = np.ascontiguousarray(coords, dtype=np.float64)
    conn = np.ascontiguousarray(conn, dtype=np.int32)
    m = fo.fo_mesh(dim, coords.shape[0], conn.shape[1], coords.ctypes.data, conn.ctypes.data,
                   None, 0, None, None)
    mat = fo.fo_material(1.0, 0.3, 1, 1e-3)
    h = C.c_void_p()
    return lib.fo_create(C.byref(h), C.byref(m), C.byref(mat), 1, None)


def test_create_rejects_bad_meshes_on_host(lib):
    from paper_2601_05709_amd import fo
    P = np.array([[0, 0], [1, 0], [0, 1]], float)
    # degenerate (collinear) triangle
    assert _create(lib, 2, np.array([[0, 0], [1, 0], [2, 0]], float), [[0], [1], [2]]) == fo.FO_ERR_MESH
    # index out of range
    assert _create(lib, 2, P, [[0], [1], [3]]) == fo.FO_ERR_MESH
    # negative index
    assert _create(lib, 2, P, [[0], [-1], [2]]) == fo.FO_ERR_MESH
    # unsupported dimension
    assert _create(lib, 4, P, [[0], [1], [2]]) == fo.FO_ERR_ARG
    # NaN coordinate -> degenerate
    assert _create(lib, 2, np.array([[0, 0], [np.nan, 0], [0, 1]], float), [[0], [1], [2]]) == fo.FO_ERR_MESH


def test_null_arguments_rejected(lib):
    from paper_2601_05709_amd import fo
    assert lib.fo_create(None, None, None, 1, None) == fo.FO_ERR_ARG
    assert lib.fo_destroy(None) == fo.FO_ERR_ARG
    assert lib.fo_state_solve(None, None, None, 1, 1, None, None) == fo.FO_ERR_ARG


def test_inverse_entries_reject_null_arguments(lib):
    from paper_2601_05709_amd import fo
    assert lib.fo_inverse_states(None, None, None, 1, 1, None, None, 10.0, 1.0, 1.0, None, None, None, None, None,
                                 None, None) == fo.FO_ERR_ARG
    assert lib.fo_inverse_derivative(None, 1, 1, None, None, None, None, None, 10.0, 1.0, None) == fo.FO_ERR_ARG


def test_loop_entries_reject_null_arguments(lib):
    from paper_2601_05709_amd import fo
    assert lib.fo_optimize(None, None, None, None, None, None, None) == fo.FO_ERR_ARG
    assert lib.fo_optimize_heat(None, None, None, None, None, None, None, None) == fo.FO_ERR_ARG
    assert lib.fo_optimize_inverse(None, None, None, 1, 1, None, None, 10.0, 1.0, 1.0, None, None, None,
                                   None) == fo.FO_ERR_ARG


def test_descent_opts_layout_and_defaults():
    from paper_2601_05709_amd import fo
    # the velocity mask is the last field of fo_descent_opts (after the boxes pointer)
    assert [f[0] for f in fo.fo_descent_opts._fields_] == ["alpha", "gamma_n", "gamma_s", "n_boxes", "boxes",
                                                            "fixed"]
    assert fo.fo_descent_opts.fixed.offset == fo.fo_descent_opts.boxes.offset + C.sizeof(C.c_void_p)
    # no boxes and no mask: an empty Omega_0 and a null mask
    for dim in (2, 3):
        d = fo.DescentOpts(alpha=0.01, gamma_n=0.0, gamma_s=0.0, dim=dim).c()
        assert d.n_boxes == 0 and not d.boxes and not d.fixed


def test_time_steps_match_oracle_rule():
    """The product's host-side time-step rule and the oracle's agree."""
    import oracle as oc
    from paper_2601_05709_amd import fo
    for B in (1e-9, 0.01, 0.3, 1.0, 7.0, 1e9):
        assert fo.time_steps(B) == pytest.approx(oc.adaptive_dt(B), rel=1e-15)


def test_workspace_bytes_on_the_host(lib):
    """fo_workspace_bytes runs fo_create's host part only: it works without a
    GPU, grows with the mesh and with the load-case block, and is 0 for an
    invalid mesh."""
    import fo_inputs as fi
    from paper_2601_05709_amd import fo

    def wsb(w, max_rhs=1, conn=None):
        m = w.mesh
        coords = np.ascontiguousarray(m.coords)
        cn = np.ascontiguousarray(m.conn if conn is None else conn, dtype=np.int32)
        bf = np.ascontiguousarray(m.bfacets, dtype=np.int32)
        bn = np.ascontiguousarray(m.bnormal)
        fx = np.ascontiguousarray(w.fixed, dtype=np.uint8)
        mesh = fo.fo_mesh(m.dim, m.n_nodes, m.n_elems, coords.ctypes.data, cn.ctypes.data, fx.ctypes.data,
                          int(bf.shape[1]), bf.ctypes.data, bn.ctypes.data)
        mat = fo.fo_material(w.E, w.nu, w.plane_stress, w.ersatz)
        return lib.fo_workspace_bytes(C.byref(mesh), C.byref(mat), max_rhs)

    small, big = fi.cantilever_3d((8, 4, 4)), fi.cantilever_3d((16, 8, 8))
    a, b = wsb(small), wsb(big)
    assert 0 < a < b and a % 256 == 0
    assert wsb(small, 20) > a
    # the same as the estimate used for admission, to the estimate's accuracy
    m = big.mesh
    est = lib.fo_footprint_estimate(C.byref(fo.fo_mesh(m.dim, m.n_nodes, m.n_elems, m.coords.ctypes.data,
                                                       np.ascontiguousarray(m.conn, dtype=np.int32).ctypes.data,
                                                       None, int(m.bfacets.shape[1]),
                                                       np.ascontiguousarray(m.bfacets, dtype=np.int32).ctypes.data,
                                                       np.ascontiguousarray(m.bnormal).ctypes.data)))
    assert 0.5 * est <= b <= 1.5 * est
    bad = np.array(small.mesh.conn, dtype=np.int32)
    bad[0, 0] = small.mesh.n_nodes  # out of range
    assert wsb(small, 1, bad) == 0


def test_time_steps_interior_value_and_errors(lib):
    """B(theta, theta) = 2 with the paper's defaults: t_end = 0.005 and
    8 (4/99)^(1/6) + 8 = 12.686 -> 13 steps (by hand)."""
    from paper_2601_05709_amd import fo
    t, s, dt = fo.time_steps(2.0)
    assert t == 0.005 and s == 13 and dt == pytest.approx(0.005 / 13, rel=1e-15)
    with pytest.raises(fo.FoError):
        fo.time_steps(1.0, dfactor=0.0)
    with pytest.raises(fo.FoError):
        fo.time_steps(1.0, s_range=(8, 4))
