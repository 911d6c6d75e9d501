"""ctypes binding of libfo (include/fo.h).

Argument marshalling only: every step of the hot path runs in the HIP
library.  Device arrays are torch tensors on the ROCm device; the binding
passes their data pointers and torch's current HIP stream.  If libfo.so is
missing the import fails loudly -- there is no CPU fallback.
"""
from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass
from typing import Optional

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libfo.so")

FO_OK, FO_NOT_CONVERGED = 0, 1
FO_ERR_ARG, FO_ERR_MESH, FO_ERR_NOMEM, FO_ERR_HIP, FO_ERR_BREAKDOWN, FO_ERR_STATE = -1, -2, -3, -4, -5, -6
FO_ERR_BUSY = -7
FO_FP64, FO_FP32_IR = 0, 1
FO_SCATTER_TILED, FO_SCATTER_ATOMIC = 0, 1


class FoError(RuntimeError):
    def __init__(self, status: int, what: str):
        super().__init__("%s: %s (status %d)" % (what, status_string(status), status))
        self.status = status


class fo_mesh(C.Structure):
    _fields_ = [("dim", C.c_int32), ("n_nodes", C.c_int64), ("n_elems", C.c_int64),
                ("coords", C.c_void_p), ("conn", C.c_void_p), ("dof_fixed", C.c_void_p),
                ("n_bfacets", C.c_int64), ("bfacets", C.c_void_p), ("bnormal", C.c_void_p)]


class fo_material(C.Structure):
    _fields_ = [("E", C.c_double), ("nu", C.c_double), ("plane_stress", C.c_int32),
                ("ersatz", C.c_double)]


class fo_solve_opts(C.Structure):
    _fields_ = [("precision", C.c_int32), ("rtol", C.c_double), ("max_iter", C.c_int32),
                ("inner_rtol", C.c_double), ("max_outer", C.c_int32), ("check_every", C.c_int32)]


class fo_descent_opts(C.Structure):
    _fields_ = [("alpha", C.c_double), ("gamma_n", C.c_double), ("gamma_s", C.c_double),
                ("n_boxes", C.c_int32), ("boxes", C.c_void_p), ("fixed", C.c_void_p)]


class fo_solve_stats(C.Structure):
    _fields_ = [("status", C.c_int32), ("iters_inner", C.c_int32), ("iters_outer", C.c_int32),
                ("rel_res", C.c_double), ("seconds", C.c_double)]


class fo_loop_opts(C.Structure):
    _fields_ = [("n_iter", C.c_int32), ("V", C.c_double), ("dfactor", C.c_double), ("t_min", C.c_double),
                ("t_max", C.c_double), ("s_min", C.c_int32), ("s_max", C.c_int32), ("smooth", C.c_int32),
                ("start_to_check", C.c_int32), ("prev", C.c_int32), ("cost_tol", C.c_double),
                ("lgrn_tol", C.c_double), ("ctrn_tol", C.c_double), ("ppl_r", C.c_double),
                ("ppl_delta0", C.c_double), ("ppl_alpha", C.c_double), ("ppl_beta", C.c_double),
                ("state", fo_solve_opts), ("descent", fo_solve_opts), ("transport", fo_solve_opts),
                ("velocity", fo_descent_opts), ("reinit_step", C.c_int32), ("reinit_iters", C.c_int32),
                ("reinit_t", C.c_double)]


class fo_loop_record(C.Structure):
    _fields_ = [("J", C.c_double), ("vol", C.c_double), ("C", C.c_double), ("L", C.c_double),
                ("lambda_", C.c_double), ("B_tt", C.c_double), ("t_end", C.c_double), ("dt", C.c_double),
                ("steps", C.c_int32), ("state_iters", C.c_int32), ("descent_iters", C.c_int32),
                ("transport_iters", C.c_int32), ("status", C.c_int32), ("reinit_iters", C.c_int32)]


_vp = C.c_void_p
class fo_request(C.Structure):
    _fields_ = [("mesh", fo_mesh), ("mat", fo_material), ("mesh_key", C.c_uint64),
                ("phi", C.c_void_p), ("b", C.c_void_p), ("state_opts", fo_solve_opts),
                ("descent_solve_opts", fo_solve_opts), ("descent", fo_descent_opts),
                ("lambda_vol", C.c_double), ("V", C.c_double), ("u_out", C.c_void_p),
                ("rhs_out", C.c_void_p), ("theta_out", C.c_void_p)]


class fo_pool_result(C.Structure):
    _fields_ = [("status", C.c_int32), ("reused_context", C.c_int32), ("state", fo_solve_stats),
                ("descent", fo_solve_stats), ("J", C.c_double), ("vol", C.c_double), ("B_tt", C.c_double),
                ("t_admit", C.c_double), ("t_start", C.c_double), ("t_end", C.c_double)]


EXPORTS = {
    "fo_create": ([C.POINTER(_vp), C.POINTER(fo_mesh), C.POINTER(fo_material), C.c_int32, _vp], C.c_int),
    "fo_create_in": ([C.POINTER(_vp), C.POINTER(fo_mesh), C.POINTER(fo_material), C.c_int32, _vp, _vp, C.c_size_t],
                     C.c_int),
    "fo_workspace_bytes": ([C.POINTER(fo_mesh), C.POINTER(fo_material), C.c_int32], C.c_size_t),
    "fo_destroy": ([_vp], C.c_int),
    "fo_footprint_bytes": ([_vp], C.c_size_t),
    "fo_set_scatter": ([_vp, C.c_int32], C.c_int),
    "fo_set_levelset": ([_vp, _vp], C.c_int),
    "fo_apply_elasticity": ([_vp, _vp, _vp, C.c_int32], C.c_int),
    "fo_state_solve": ([_vp, _vp, _vp, C.c_int32, C.c_int64, C.POINTER(fo_solve_opts),
                        C.POINTER(fo_solve_stats)], C.c_int),
    "fo_shape_derivative": ([_vp, _vp, C.c_int32, C.c_int64, C.c_double, C.c_double, _vp, _vp,
                             _vp, _vp], C.c_int),
    "fo_descent_solve": ([_vp, C.POINTER(fo_descent_opts), _vp, _vp, C.POINTER(fo_solve_opts),
                          C.POINTER(fo_solve_stats), _vp], C.c_int),
    "fo_apply_descent": ([_vp, C.POINTER(fo_descent_opts), _vp, _vp], C.c_int),
    "fo_levelset_update": ([_vp, _vp, C.c_double, _vp], C.c_int),
    "fo_heat_load": ([_vp, _vp, _vp], C.c_int),
    "fo_heat_solve": ([_vp, _vp, _vp, _vp, C.POINTER(fo_solve_opts), C.POINTER(fo_solve_stats)], C.c_int),
    "fo_heat_derivative": ([_vp, _vp, _vp, C.c_double, C.c_double, _vp, _vp, _vp], C.c_int),
    "fo_inverse_states": ([_vp, _vp, _vp, C.c_int32, C.c_int64, _vp, _vp, C.c_double, C.c_double, C.c_double,
                           C.POINTER(fo_solve_opts), _vp, _vp, _vp, _vp, _vp, C.POINTER(fo_solve_stats)], C.c_int),
    "fo_inverse_derivative": ([_vp, C.c_int32, C.c_int64, _vp, _vp, _vp, _vp, _vp, C.c_double, C.c_double, _vp],
                              C.c_int),
    "fo_reinit": ([_vp, _vp, C.c_int32, C.c_double, C.POINTER(fo_solve_opts), C.POINTER(fo_solve_stats)],
                  C.c_int),
    "fo_optimize": ([_vp, C.POINTER(fo_loop_opts), _vp, _vp, C.POINTER(fo_loop_record), C.POINTER(C.c_int32),
                     C.POINTER(C.c_int32)], C.c_int),
    "fo_optimize_noalloc": ([_vp, C.POINTER(fo_loop_opts), _vp, _vp, C.POINTER(fo_loop_record),
                             C.POINTER(C.c_int32), C.POINTER(C.c_int32)], C.c_int),
    "fo_device_allocations": ([], C.c_int64),
    "fo_optimize_heat": ([_vp, C.POINTER(fo_loop_opts), _vp, _vp, _vp, C.POINTER(fo_loop_record),
                          C.POINTER(C.c_int32), C.POINTER(C.c_int32)], C.c_int),
    "fo_optimize_inverse": ([_vp, _vp, C.POINTER(fo_loop_opts), C.c_int32, C.c_int64, _vp, _vp, C.c_double,
                             C.c_double, C.c_double, _vp, C.POINTER(fo_loop_record), C.POINTER(C.c_int32),
                             C.POINTER(C.c_int32)], C.c_int),
    "fo_transport": ([_vp, _vp, C.c_double, C.c_int32, C.c_int32, _vp, C.POINTER(fo_solve_opts),
                      C.POINTER(fo_solve_stats)], C.c_int),
    "fo_profile_enable": ([_vp, C.c_int32], C.c_int),
    "fo_profile_read": ([_vp, C.c_int32, C.POINTER(C.c_double), C.POINTER(C.c_int64)], C.c_int),
    "fo_time_kernel": ([_vp, C.c_int32, C.c_int32, C.POINTER(C.c_double)], C.c_int),
    "fo_batch_tune": ([_vp, C.c_int32, C.POINTER(C.c_int32), C.POINTER(C.c_int32), C.POINTER(C.c_double)],
                      C.c_int),
    "fo_apply_elasticity_batch": ([_vp, _vp, _vp, C.c_int32], C.c_int),
    "fo_set_batch_method": ([_vp, C.c_int32], C.c_int),
    "fo_set_batch_operator": ([_vp, C.c_int32], C.c_int),
    "fo_nodal_stats": ([_vp, C.POINTER(C.c_int32), C.POINTER(C.c_int64), C.POINTER(C.c_int64)], C.c_int),
    "fo_batch_stats": ([_vp, C.POINTER(C.c_int32), C.POINTER(C.c_int32), C.POINTER(C.c_int32),
                        C.POINTER(C.c_int64), C.POINTER(C.c_int64)], C.c_int),
    "fo_tile_stats": ([_vp] + [C.POINTER(C.c_int64)] * 5, C.c_int),
    "fo_footprint_estimate": ([C.POINTER(fo_mesh)], C.c_size_t),
    "fo_pool_create": ([C.POINTER(_vp), C.c_size_t, C.c_int32], C.c_int),
    "fo_pool_admit": ([_vp, C.POINTER(fo_request), C.POINTER(C.c_int32)], C.c_int),
    "fo_pool_step": ([_vp, C.POINTER(C.c_int32)], C.c_int),
    "fo_pool_wait": ([_vp, C.c_int64, C.POINTER(C.c_int32)], C.c_int),
    "fo_pool_poll": ([_vp, C.c_int32, C.POINTER(C.c_int32), C.POINTER(fo_pool_result)], C.c_int),
    "fo_pool_release": ([_vp, C.c_int32], C.c_int),
    "fo_pool_stats": ([_vp, C.POINTER(C.c_size_t), C.POINTER(C.c_int32), C.POINTER(C.c_int32)], C.c_int),
    "fo_pool_destroy": ([_vp], C.c_int),
    "fo_status_string": ([C.c_int], C.c_char_p),
    "fo_time_steps": ([C.c_double, C.c_double, C.c_double, C.c_double, C.c_int32, C.c_int32, C.POINTER(C.c_double),
                       C.POINTER(C.c_int32), C.POINTER(C.c_double)], C.c_int),
}

FO_PROF_ELAS_TILE_FP64, FO_PROF_ELAS_TILE_FP32, FO_PROF_HALO_FP64, FO_PROF_HALO_FP32 = 0, 1, 2, 3
FO_KERNEL_CG_OP_FP64, FO_KERNEL_CG_OP_FP32, FO_KERNEL_BATCH_APPLY = 0, 1, 2
FO_BATCH_BLOCK_CG, FO_BATCH_COLUMN_CG = 0, 1
FO_BATCH_OP_NODAL, FO_BATCH_OP_ELEMENT = 0, 1
FO_NOALLOC_MAX_DOFS = 2796201  # largest n_dofs of fo_optimize_noalloc (include/fo.h)

_lib = None


def lib():
    """Loads libfo.so (built in-tree by build()); raises if it is missing."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError("libfo.so is not built (%s); run __graft_entry__.build() or "
                               "python -m paper_2601_05709_amd.build" % LIB_PATH)
        L = C.CDLL(LIB_PATH)
        for name, (args, res) in EXPORTS.items():
            f = getattr(L, name)
            f.argtypes = args
            f.restype = res
        _lib = L
    return _lib


def device_allocations() -> int:
    """Device allocations the library has made in this process (fo_device_allocations)."""
    return int(lib().fo_device_allocations())


def status_string(s: int) -> str:
    try:
        return lib().fo_status_string(int(s)).decode()
    except Exception:  # library not loadable: still format the error
        return "status %d" % s


def _check(rc: int, what: str, allow=(FO_OK,)) -> int:
    if rc not in allow:
        raise FoError(rc, what)
    return rc


def _ptr(t, dtype=None, numel=None, name="array"):
    """Device pointer of a contiguous torch tensor (validated), or None."""
    if t is None:
        return None
    import torch
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError("%s must be a torch tensor on the GPU" % name)
    if not t.is_contiguous():
        raise ValueError("%s must be contiguous" % name)
    if dtype is not None and t.dtype != dtype:
        raise TypeError("%s must have dtype %s (got %s)" % (name, dtype, t.dtype))
    if numel is not None and t.numel() < numel:
        raise ValueError("%s has %d elements, needs %d" % (name, t.numel(), numel))
    return C.c_void_p(t.data_ptr())


@dataclass
class SolveOpts:
    precision: int = FO_FP64
    rtol: float = 1e-8
    max_iter: int = 200000
    inner_rtol: float = 0.1
    max_outer: int = 60
    check_every: int = 0

    def c(self) -> fo_solve_opts:
        return fo_solve_opts(self.precision, self.rtol, self.max_iter, self.inner_rtol,
                             self.max_outer, self.check_every)


@dataclass
class Stats:
    status: int
    iters_inner: int
    iters_outer: int
    rel_res: float
    seconds: float


class DescentOpts:
    def __init__(self, alpha=0.01, gamma_n=1e4, gamma_s=1e4, boxes=None, dim=None, fixed=None):
        """fixed: optional device uint8 tensor [n_dofs]; theta = 0 where it is set."""
        self.alpha, self.gamma_n, self.gamma_s = float(alpha), float(gamma_n), float(gamma_s)
        self.fixed = fixed
        b = np.zeros((0, 2 * (dim or 2))) if boxes is None else np.asarray(boxes, dtype=np.float64)
        self.boxes = np.ascontiguousarray(b.reshape(b.shape[0], -1) if b.size else b.reshape(0, 2 * (dim or 2)))

    def c(self, n_dofs: Optional[int] = None) -> fo_descent_opts:
        """The C struct; with n_dofs, the mask is checked to hold that many entries."""
        n = self.boxes.shape[0]
        ptr = self.boxes.ctypes.data_as(C.c_void_p) if n else None
        fx = None
        if self.fixed is not None:
            import torch
            fx = _ptr(self.fixed, torch.uint8, n_dofs, "fixed")
        return fo_descent_opts(self.alpha, self.gamma_n, self.gamma_s, n, ptr, fx)


def current_stream():
    import torch
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


class Context:
    """One mesh + material resident on the GPU (fo_create / fo_destroy)."""

    def __init__(self, dim, coords, conn, fixed=None, bfacets=None, bnormal=None, E=1.0, nu=0.3,
                 plane_stress=1, ersatz=1e-3, max_rhs=1, stream=None, workspace=False):
        """workspace: the context's device arrays are carved from one caller-owned
        buffer of fo_workspace_bytes bytes (a torch tensor held here; fo_create_in)
        instead of allocated by the library (fo_create)."""
        L = lib()
        self.dim = int(dim)
        self._coords = np.ascontiguousarray(coords, dtype=np.float64)
        self._conn = np.ascontiguousarray(conn, dtype=np.int32)
        self.n_nodes = int(self._coords.shape[0])
        self.n_elems = int(self._conn.shape[1])
        self.n_dofs = self.n_nodes * self.dim
        self.max_rhs = int(max_rhs)
        fx = None if fixed is None else np.ascontiguousarray(fixed, dtype=np.uint8)
        bf = None if bfacets is None else np.ascontiguousarray(bfacets, dtype=np.int32)
        bn = None if bnormal is None else np.ascontiguousarray(bnormal, dtype=np.float64)
        if fx is not None and fx.size != self.n_dofs:
            raise ValueError("fixed must have n_nodes*dim entries")
        nbf = 0 if bf is None else int(bf.shape[1])
        m = fo_mesh(self.dim, self.n_nodes, self.n_elems, self._coords.ctypes.data, self._conn.ctypes.data,
                    None if fx is None else fx.ctypes.data, nbf,
                    None if bf is None else bf.ctypes.data, None if bn is None else bn.ctypes.data)
        mat = fo_material(E, nu, int(plane_stress), ersatz)
        h = C.c_void_p()
        self.stream = stream if stream is not None else current_stream()
        self.ws = None
        if workspace:
            import torch
            nb = int(L.fo_workspace_bytes(C.byref(m), C.byref(mat), self.max_rhs))
            if nb == 0:
                raise FoError(FO_ERR_ARG, "fo_workspace_bytes")
            self.ws = torch.empty(nb, dtype=torch.uint8, device="cuda")
            _check(L.fo_create_in(C.byref(h), C.byref(m), C.byref(mat), self.max_rhs, self.stream,
                                  C.c_void_p(self.ws.data_ptr()), nb), "fo_create_in")
        else:
            _check(L.fo_create(C.byref(h), C.byref(m), C.byref(mat), self.max_rhs, self.stream), "fo_create")
        self.h = h

    @classmethod
    def from_workload(cls, w, max_rhs=None, stream=None, workspace=False):
        m = w.mesh
        return cls(m.dim, m.coords, m.conn, w.fixed, m.bfacets, m.bnormal, w.E, w.nu, w.plane_stress,
                   w.ersatz, max_rhs or w.n_rhs, stream, workspace)

    def close(self):
        if getattr(self, "h", None):
            lib().fo_destroy(self.h)
            self.h = None
        self.ws = None  # the workspace outlives the context it backs

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def footprint(self) -> int:
        return int(lib().fo_footprint_bytes(self.h))

    def profile_enable(self, on: bool = True):
        _check(lib().fo_profile_enable(self.h, 1 if on else 0), "fo_profile_enable")

    def profile_read(self, which: int):
        ms, n = C.c_double(), C.c_int64()
        _check(lib().fo_profile_read(self.h, which, C.byref(ms), C.byref(n)), "fo_profile_read")
        return ms.value, n.value

    def time_kernel(self, kernel: int, reps: int = 200) -> float:
        """Average duration (us) of `reps` back-to-back launches of a kernel
        (fo_time_kernel); clobbers the CG work vectors."""
        us = C.c_double()
        _check(lib().fo_time_kernel(self.h, kernel, reps, C.byref(us)), "fo_time_kernel")
        return us.value

    def tile_stats(self) -> dict:
        v = [C.c_int64() for _ in range(5)]
        _check(lib().fo_tile_stats(self.h, *[C.byref(x) for x in v]), "fo_tile_stats")
        keys = ("n_tiles", "max_nodes", "n_slots", "n_shared_nodes", "n_halo_slots")
        return dict(zip(keys, (x.value for x in v)))

    def set_scatter(self, mode: int):
        _check(lib().fo_set_scatter(self.h, mode), "fo_set_scatter")

    def set_levelset(self, phi):
        import torch
        _check(lib().fo_set_levelset(self.h, _ptr(phi, torch.float64, self.n_nodes, "phi")),
               "fo_set_levelset")

    def apply_elasticity(self, x, y, precision=FO_FP64):
        import torch
        dt = torch.float64 if precision == FO_FP64 else torch.float32
        _check(lib().fo_apply_elasticity(self.h, _ptr(x, dt, self.n_dofs, "x"),
                                         _ptr(y, dt, self.n_dofs, "y"), precision),
               "fo_apply_elasticity")

    def apply_elasticity_batch(self, x, y, ncols: int):
        """y = K(phi) x on FP32 blocks [n_dofs][ncols] (batched operator)."""
        import torch
        _check(lib().fo_apply_elasticity_batch(self.h, _ptr(x, torch.float32, self.n_dofs * ncols, "x"),
                                               _ptr(y, torch.float32, self.n_dofs * ncols, "y"), ncols),
               "fo_apply_elasticity_batch")

    def batch_tune(self, n_rhs: int):
        """Picks the batch tile node cap and register group size with the
        fastest batched apply; returns (node cap, group, apply microseconds)."""
        nodes, group, us = C.c_int32(), C.c_int32(), C.c_double()
        _check(lib().fo_batch_tune(self.h, n_rhs, C.byref(nodes), C.byref(group), C.byref(us)),
               "fo_batch_tune")
        return nodes.value, group.value, us.value

    def set_batch_method(self, method: int):
        """Solver of the batched multi-load solves: FO_BATCH_COLUMN_CG (CG per
        column, the default) or FO_BATCH_BLOCK_CG (block CG)."""
        _check(lib().fo_set_batch_method(self.h, int(method)), "fo_set_batch_method")

    def nodal_stats(self) -> dict:
        """Assembled operator of the batched path: neighbour slots per node,
        off-diagonal blocks and device bytes (zeros when absent)."""
        nb, od, by = C.c_int32(), C.c_int64(), C.c_int64()
        _check(lib().fo_nodal_stats(self.h, C.byref(nb), C.byref(od), C.byref(by)), "fo_nodal_stats")
        return {"slots": nb.value, "off_diagonal_blocks": od.value, "bytes": by.value}

    def set_batch_operator(self, op: int):
        """Operator of the batched solves: FO_BATCH_OP_NODAL (assembled node
        blocks, the default) or FO_BATCH_OP_ELEMENT (element tiles)."""
        _check(lib().fo_set_batch_operator(self.h, int(op)), "fo_set_batch_operator")

    def batch_stats(self) -> dict:
        cols, nodes, group = C.c_int32(), C.c_int32(), C.c_int32()
        nt, hs = C.c_int64(), C.c_int64()
        _check(lib().fo_batch_stats(self.h, C.byref(cols), C.byref(nodes), C.byref(group), C.byref(nt),
                                    C.byref(hs)), "fo_batch_stats")
        return {"columns": cols.value, "tile_nodes": nodes.value, "group": group.value,
                "n_tiles": nt.value, "n_halo_slots": hs.value}

    def state_solve(self, b, u, opts: SolveOpts, n_rhs: int = 1, ld: Optional[int] = None,
                    allow_not_converged=False) -> Stats:
        import torch
        ld = n_rhs if ld is None else ld
        st = fo_solve_stats()
        allow = (FO_OK, FO_NOT_CONVERGED) if allow_not_converged else (FO_OK,)
        rc = lib().fo_state_solve(self.h, _ptr(b, torch.float64, self.n_dofs * ld, "b"),
                                  _ptr(u, torch.float64, self.n_dofs * ld, "u"), n_rhs, ld,
                                  C.byref(opts.c()), C.byref(st))
        _check(rc, "fo_state_solve", allow)
        return Stats(st.status, st.iters_inner, st.iters_outer, st.rel_res, st.seconds)

    def shape_derivative(self, u, rhs, J, vol, n_rhs=1, ld=None, lambda_vol=0.0, V=1.0, S1=None):
        import torch
        ld = n_rhs if ld is None else ld
        _check(lib().fo_shape_derivative(
            self.h, _ptr(u, torch.float64, self.n_dofs * ld, "u"), n_rhs, ld, lambda_vol, V,
            _ptr(rhs, torch.float64, self.n_dofs, "rhs"),
            _ptr(S1, torch.float64, self.dim * self.dim * self.n_elems, "S1"),
            _ptr(J, torch.float64, n_rhs, "J"), _ptr(vol, torch.float64, 1, "vol")),
            "fo_shape_derivative")

    def descent_solve(self, dopts: DescentOpts, rhs, theta, opts: SolveOpts, B_tt=None,
                      allow_not_converged=False) -> Stats:
        import torch
        st = fo_solve_stats()
        allow = (FO_OK, FO_NOT_CONVERGED) if allow_not_converged else (FO_OK,)
        rc = lib().fo_descent_solve(self.h, C.byref(dopts.c(self.n_dofs)),
                                    _ptr(rhs, torch.float64, self.n_dofs, "rhs"),
                                    _ptr(theta, torch.float64, self.n_dofs, "theta"),
                                    C.byref(opts.c()), C.byref(st),
                                    _ptr(B_tt, torch.float64, 1, "B_tt"))
        _check(rc, "fo_descent_solve", allow)
        return Stats(st.status, st.iters_inner, st.iters_outer, st.rel_res, st.seconds)

    def apply_descent(self, dopts: DescentOpts, x, y):
        import torch
        _check(lib().fo_apply_descent(self.h, C.byref(dopts.c(self.n_dofs)), _ptr(x, torch.float64, self.n_dofs, "x"),
                                      _ptr(y, torch.float64, self.n_dofs, "y")), "fo_apply_descent")

    def transport(self, theta, dt: float, steps: int, phi, opts: Optional[SolveOpts] = None,
                  smooth: bool = True, allow_not_converged=False) -> Stats:
        """The paper's transport step: `steps` Crank-Nicolson Petrov-Galerkin
        steps of length dt (fo_transport); phi is updated in place."""
        import torch
        opts = opts or SolveOpts(rtol=1e-10)
        st = fo_solve_stats()
        allow = (FO_OK, FO_NOT_CONVERGED) if allow_not_converged else (FO_OK,)
        rc = lib().fo_transport(self.h, _ptr(theta, torch.float64, self.n_dofs, "theta"), float(dt), int(steps),
                                int(bool(smooth)), _ptr(phi, torch.float64, self.n_nodes, "phi"),
                                C.byref(opts.c()), C.byref(st))
        _check(rc, "fo_transport", allow)
        return Stats(st.status, st.iters_inner, st.iters_outer, st.rel_res, st.seconds)

    def heat_load(self, f, b):
        """b = int f lambda_a for the nodal heat source f (fo_heat_load)."""
        import torch
        _check(lib().fo_heat_load(self.h, _ptr(f, torch.float64, self.n_nodes, "f"),
                                  _ptr(b, torch.float64, self.n_nodes, "b")), "fo_heat_load")

    def heat_solve(self, gamma0, b, u, opts: Optional[SolveOpts] = None, allow_not_converged=False) -> Stats:
        """Heat state u (fo_heat_solve): K u = b, u = 0 where gamma0 (uint8 [N]) is set."""
        import torch
        opts = opts or SolveOpts(rtol=1e-10)
        st = fo_solve_stats()
        rc = lib().fo_heat_solve(self.h, _ptr(gamma0, torch.uint8, self.n_nodes, "gamma0"),
                                 _ptr(b, torch.float64, self.n_nodes, "b"), _ptr(u, torch.float64, self.n_nodes, "u"),
                                 C.byref(opts.c()), C.byref(st))
        _check(rc, "fo_heat_solve", (FO_OK, FO_NOT_CONVERGED) if allow_not_converged else (FO_OK,))
        return Stats(st.status, st.iters_inner, st.iters_outer, st.rel_res, st.seconds)

    def heat_derivative(self, u, f, rhs, J, vol, lambda_vol=0.0, V=1.0):
        """Descent right-hand side, cost and volume of the heat model (fo_heat_derivative)."""
        import torch
        _check(lib().fo_heat_derivative(self.h, _ptr(u, torch.float64, self.n_nodes, "u"),
                                        _ptr(f, torch.float64, self.n_nodes, "f"), float(lambda_vol), float(V),
                                        _ptr(rhs, torch.float64, self.n_dofs, "rhs"), _ptr(J, torch.float64, 1, "J"),
                                        _ptr(vol, torch.float64, 1, "vol")), "fo_heat_derivative")

    def inverse_states(self, ctx_g: "Context", phi, f, g, kappa: float, alpha: float, beta: float, u, v, p, q, J,
                       opts: Optional[SolveOpts] = None, n_pairs: int = 1, ld: Optional[int] = None,
                       allow_not_converged=False) -> Stats:
        """States u, v, adjoints p, q and the cost J [n_pairs] of the inverse
        elasticity problem (fo_inverse_states) for n_pairs pairs stored as
        columns of [n_dofs][ld] arrays; self clamps Gamma_0, ctx_g the whole
        boundary, both with ersatz = 1/kappa."""
        import torch
        opts = opts or SolveOpts(precision=FO_FP64, rtol=1e-10)
        ld = n_pairs if ld is None else ld
        st = fo_solve_stats()
        n = self.n_dofs * ld
        rc = lib().fo_inverse_states(self.h, ctx_g.h, _ptr(phi, torch.float64, self.n_nodes, "phi"), int(n_pairs),
                                     int(ld), _ptr(f, torch.float64, n, "f"), _ptr(g, torch.float64, n, "g"),
                                     float(kappa), float(alpha), float(beta), C.byref(opts.c()),
                                     _ptr(u, torch.float64, n, "u"), _ptr(v, torch.float64, n, "v"),
                                     _ptr(p, torch.float64, n, "p"), _ptr(q, torch.float64, n, "q"),
                                     _ptr(J, torch.float64, n_pairs, "J"), C.byref(st))
        _check(rc, "fo_inverse_states", (FO_OK, FO_NOT_CONVERGED) if allow_not_converged else (FO_OK,))
        return Stats(st.status, st.iters_inner, st.iters_outer, st.rel_res, st.seconds)

    def inverse_derivative(self, u, v, p, q, g, kappa: float, alpha: float, rhs, n_pairs: int = 1,
                           ld: Optional[int] = None):
        """Descent right-hand side of the inverse problem summed over the
        pairs (fo_inverse_derivative)."""
        import torch
        ld = n_pairs if ld is None else ld
        n = self.n_dofs * ld
        _check(lib().fo_inverse_derivative(self.h, int(n_pairs), int(ld),
                                           *(_ptr(x, torch.float64, n, nm) for x, nm in
                                             ((u, "u"), (v, "v"), (p, "p"), (q, "q"), (g, "g"))),
                                           float(kappa), float(alpha), _ptr(rhs, torch.float64, self.n_dofs, "rhs")),
               "fo_inverse_derivative")

    def reinit(self, phi, steps: int = 8, t_end: float = 0.1, opts: Optional[SolveOpts] = None,
               allow_not_converged=False) -> Stats:
        """Reinitialisation of the level set (fo_reinit): `steps` pseudo-time
        steps of the diffusive Eikonal equation up to t_end; phi in place."""
        import torch
        opts = opts or SolveOpts(rtol=1e-10)
        st = fo_solve_stats()
        rc = lib().fo_reinit(self.h, _ptr(phi, torch.float64, self.n_nodes, "phi"), int(steps), float(t_end),
                             C.byref(opts.c()), C.byref(st))
        _check(rc, "fo_reinit", (FO_OK, FO_NOT_CONVERGED) if allow_not_converged else (FO_OK,))
        return Stats(st.status, st.iters_inner, st.iters_outer, st.rel_res, st.seconds)

    def optimize(self, b, phi, n_iter: int, dopts: "DescentOpts", V: Optional[float] = None, smooth=False,
                 dfactor=1e-2, lv_time=(1e-3, 1e-1), lv_iter=(8, 16), start_to_check=30, prev=10,
                 cost_tol=1e-2, lgrn_tol=1e-2, ctrn_tol=1e-2, ppl=(0.999, 0.5, 2000.0, 0.5),
                 state_opts: Optional[SolveOpts] = None, descent_opts: Optional[SolveOpts] = None,
                 transport_opts: Optional[SolveOpts] = None, reinit_step=0, reinit_pars=(8, 0.1),
                 allow_not_converged=False, noalloc=False):
        """The level-set loop (fo_optimize): up to n_iter iterations of the
        paper's Algorithm 1 from phi (updated in place) with the load b;
        V given: volume constraint vol / V = 1 by the PPL method.  noalloc:
        the variant without device allocation (fo_optimize_noalloc).  Returns
        (records as dicts, stopped)."""
        import torch
        o = _loop_opts(n_iter, V, smooth, dfactor, lv_time, lv_iter, start_to_check, prev, cost_tol, lgrn_tol,
                       ctrn_tol, ppl, state_opts, descent_opts, transport_opts, dopts, reinit_step, reinit_pars,
                       n_dofs=self.n_dofs)
        recs = (fo_loop_record * max(1, int(n_iter)))()
        n_done, stopped = C.c_int32(0), C.c_int32(0)
        name = "fo_optimize_noalloc" if noalloc else "fo_optimize"
        rc = getattr(lib(), name)(self.h, C.byref(o), _ptr(b, torch.float64, self.n_dofs, "b"),
                                  _ptr(phi, torch.float64, self.n_nodes, "phi"), recs, C.byref(n_done),
                                  C.byref(stopped))
        _check(rc, name, (FO_OK, FO_NOT_CONVERGED) if allow_not_converged else (FO_OK,))
        return _records(recs, n_done.value), bool(stopped.value)

    def optimize_heat(self, gamma0, f, phi, n_iter: int, dopts: "DescentOpts", V: Optional[float] = None,
                      smooth=False, dfactor=1e-2, lv_time=(1e-3, 1e-1), lv_iter=(8, 16), start_to_check=30, prev=10,
                      cost_tol=1e-2, lgrn_tol=1e-2, ctrn_tol=1e-2, ppl=(0.999, 0.5, 2000.0, 0.5),
                      state_opts: Optional[SolveOpts] = None, descent_opts: Optional[SolveOpts] = None,
                      transport_opts: Optional[SolveOpts] = None, reinit_step=0, reinit_pars=(8, 0.1),
                      allow_not_converged=False):
        """Algorithm 1 on the heat-conduction model (fo_optimize_heat):
        gamma0 uint8 [N] (u = 0 there), f the P1 source [N]; V given: volume
        constraint by the PPL method.  phi is updated in place.  Returns
        (records as dicts, stopped)."""
        import torch
        o = _loop_opts(n_iter, V, smooth, dfactor, lv_time, lv_iter, start_to_check, prev, cost_tol, lgrn_tol,
                       ctrn_tol, ppl, state_opts or SolveOpts(rtol=1e-8), descent_opts, transport_opts, dopts,
                       reinit_step, reinit_pars, n_dofs=self.n_dofs)
        recs = (fo_loop_record * max(1, int(n_iter)))()
        n_done, stopped = C.c_int32(0), C.c_int32(0)
        rc = lib().fo_optimize_heat(self.h, C.byref(o), _ptr(gamma0, torch.uint8, self.n_nodes, "gamma0"),
                                    _ptr(f, torch.float64, self.n_nodes, "f"),
                                    _ptr(phi, torch.float64, self.n_nodes, "phi"), recs, C.byref(n_done),
                                    C.byref(stopped))
        _check(rc, "fo_optimize_heat", (FO_OK, FO_NOT_CONVERGED) if allow_not_converged else (FO_OK,))
        return _records(recs, n_done.value), bool(stopped.value)

    def optimize_inverse(self, ctx_g: "Context", f, g, kappa: float, alpha: float, beta: float, phi, n_iter: int,
                         dopts: "DescentOpts", n_pairs: int = 1, ld: Optional[int] = None, smooth=False,
                         dfactor=1e-2, lv_time=(1e-3, 1e-1), lv_iter=(8, 16), start_to_check=30, prev=10,
                         cost_tol=1e-2, state_opts: Optional[SolveOpts] = None,
                         descent_opts: Optional[SolveOpts] = None, transport_opts: Optional[SolveOpts] = None,
                         reinit_step=0, reinit_pars=(8, 0.1), allow_not_converged=False):
        """Algorithm 1 on the inverse problem (fo_optimize_inverse): self
        clamps Gamma_0, ctx_g the whole boundary (both with ersatz 1/kappa);
        f, g hold n_pairs columns of [n_dofs][ld]; dopts is the velocity form
        (the paper's H^1_0 setting: fixed = the boundary unknowns).  phi is
        updated in place.  Returns (records as dicts, stopped)."""
        import torch
        ld = n_pairs if ld is None else ld
        o = _loop_opts(n_iter, None, smooth, dfactor, lv_time, lv_iter, start_to_check, prev, cost_tol, 1e-2,
                       1e-2, (0.999, 0.5, 2000.0, 0.5), state_opts, descent_opts, transport_opts, dopts,
                       reinit_step, reinit_pars, n_dofs=self.n_dofs)
        recs = (fo_loop_record * max(1, int(n_iter)))()
        n_done, stopped = C.c_int32(0), C.c_int32(0)
        n = self.n_dofs * ld
        rc = lib().fo_optimize_inverse(self.h, ctx_g.h, C.byref(o), int(n_pairs), int(ld),
                                       _ptr(f, torch.float64, n, "f"), _ptr(g, torch.float64, n, "g"), float(kappa),
                                       float(alpha), float(beta), _ptr(phi, torch.float64, self.n_nodes, "phi"),
                                       recs, C.byref(n_done), C.byref(stopped))
        _check(rc, "fo_optimize_inverse", (FO_OK, FO_NOT_CONVERGED) if allow_not_converged else (FO_OK,))
        return _records(recs, n_done.value), bool(stopped.value)

    def levelset_update(self, theta, dt: float, phi):
        import torch
        _check(lib().fo_levelset_update(self.h, _ptr(theta, torch.float64, self.n_dofs, "theta"),
                                        float(dt), _ptr(phi, torch.float64, self.n_nodes, "phi")),
               "fo_levelset_update")


def _loop_opts(n_iter, V, smooth, dfactor, lv_time, lv_iter, start_to_check, prev, cost_tol, lgrn_tol, ctrn_tol,
               ppl, state_opts, descent_opts, transport_opts, dopts, reinit_step, reinit_pars,
               n_dofs=None) -> fo_loop_opts:
    so = state_opts or SolveOpts(precision=FO_FP32_IR, rtol=1e-8)
    do = descent_opts or SolveOpts(precision=FO_FP32_IR, rtol=1e-8)
    to = transport_opts or SolveOpts(rtol=1e-10)
    return fo_loop_opts(int(n_iter), float(V) if V else 0.0, float(dfactor), float(lv_time[0]), float(lv_time[1]),
                        int(lv_iter[0]), int(lv_iter[1]), int(bool(smooth)), int(start_to_check), int(prev),
                        float(cost_tol), float(lgrn_tol), float(ctrn_tol), float(ppl[0]), float(ppl[1]),
                        float(ppl[2]), float(ppl[3]), so.c(), do.c(), to.c(), dopts.c(n_dofs), int(reinit_step or 0),
                        int(reinit_pars[0]), float(reinit_pars[1]))


def _records(recs, n):
    out = []
    for r in recs[:n]:
        d = {k: getattr(r, k) for k, _ in fo_loop_record._fields_}
        d["lambda"] = d.pop("lambda_")
        out.append(d)
    return out


def time_steps(B_tt: float, dfactor=1e-2, t_range=(1e-3, 1e-1), s_range=(8, 16)):
    """(t_end, steps, dt) of the transport from B(theta, theta) (fo_time_steps)."""
    t_end, steps, dt = C.c_double(), C.c_int32(), C.c_double()
    _check(lib().fo_time_steps(float(B_tt), float(dfactor), float(t_range[0]), float(t_range[1]),
                               int(s_range[0]), int(s_range[1]), C.byref(t_end), C.byref(steps), C.byref(dt)),
           "fo_time_steps")
    return t_end.value, steps.value, dt.value
