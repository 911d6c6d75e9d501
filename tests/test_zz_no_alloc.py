"""fo_optimize_noalloc (the level-set loop with its work vectors in the
library's static device array, no device allocation) gives the results of
fo_optimize, on two calls in a row with the second on a smaller mesh, and
allocates nothing during the call."""
import numpy as np
import pytest

import fo_inputs as fi

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from paper_2601_05709_amd import fo  # noqa: E402


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).cuda()


def loop(ctx, w, noalloc, n_iter=3):
    dopts = fo.DescentOpts(w.alpha, w.gamma_n, w.gamma_s, w.boxes, dim=w.mesh.dim)
    phi = dev(w.phi)
    V = 1.5  # a volume target: the PPL multiplier is active
    before = fo.device_allocations()
    recs, stopped = ctx.optimize(dev(w.b.reshape(-1)), phi, n_iter, dopts, V=V, noalloc=noalloc)
    torch.cuda.synchronize()
    return recs, phi.cpu().numpy(), fo.device_allocations() - before


def same(a, b):
    ra, pa, _ = a
    rb, pb, _ = b
    assert len(ra) == len(rb) > 0
    for x, y in zip(ra, rb):
        for k in ("J", "vol", "C", "L", "lambda", "B_tt", "t_end", "dt"):
            assert (x[k] == y[k]) or (np.isnan(x[k]) and np.isnan(y[k])), (k, x[k], y[k])
        for k in ("steps", "state_iters", "descent_iters", "transport_iters", "status"):
            assert x[k] == y[k], (k, x[k], y[k])
    assert np.array_equal(pa, pb)


@pytest.mark.parametrize("big,small", [((64, 32), (24, 12))])
def test_noalloc_loop_matches_fo_optimize(big, small):
    for cells in (big, small):  # two calls in a row, the second on a smaller mesh
        w = fi.cantilever_2d(cells)
        print("noalloc loop, 2D %dx%d" % cells, flush=True)
        ctx_a = fo.Context.from_workload(w)     # no captured graphs yet: direct launches
        got = loop(ctx_a, w, noalloc=True)
        assert got[2] == 0, "fo_optimize_noalloc allocated device memory"
        ctx_b = fo.Context.from_workload(w)
        ref = loop(ctx_b, w, noalloc=False)
        assert ref[2] >= 1                       # fo_optimize allocates its work vectors
        same(got, ref)
        again = loop(ctx_b, w, noalloc=True)     # a context with captured graphs
        assert again[2] == 0
        same(again, ref)
        ctx_a.close()
        ctx_b.close()


def test_noalloc_loop_rejects_meshes_beyond_its_array():
    assert (3 * fo.FO_NOALLOC_MAX_DOFS + 4) * 8 <= 64 << 20 < (3 * fo.FO_NOALLOC_MAX_DOFS + 7) * 8
    w = fi.cantilever_2d((1700, 850))  # 2,895,102 unknowns
    assert w.mesh.n_nodes * 2 > fo.FO_NOALLOC_MAX_DOFS
    print("noalloc loop, 2D 1700x850 (beyond the array)", flush=True)
    ctx = fo.Context.from_workload(w)
    phi = dev(w.phi)
    with pytest.raises(fo.FoError):
        loop(ctx, w, noalloc=True)
    np.testing.assert_array_equal(phi.cpu().numpy(), w.phi)
    ctx.close()
