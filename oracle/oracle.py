"""Python face of the FP64 CPU oracle (fo_oracle.c).

TEST INFRASTRUCTURE ONLY: imported by tests/, by the smoke check and by the
benchmark's cpu_baseline leg -- never by the product path.  It shares no code
with the HIP library.

Every routine is a thin ctypes call into fo_oracle.c plus numpy glue; the
arithmetic (element matrices, assembly, Jacobi-PCG, shape derivative,
level-set update) is in the C file, written from the paper's definitions.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
import time
from dataclasses import dataclass
from typing import Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "fo_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

_i64 = C.c_int64
_dp = C.POINTER(C.c_double)
_ip32 = C.POINTER(C.c_int32)
_ip64 = C.POINTER(C.c_int64)
_up8 = C.POINTER(C.c_uint8)


def build(force: bool = False) -> str:
    """Compile fo_oracle.c into liboracle.so with gcc (-O2, OpenMP)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-std=c11",
                               "-Wall", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        build()
        L = C.CDLL(_LIB)
        L.oc_lame.argtypes = [C.c_double, C.c_double, C.c_int, C.c_int, _dp, _dp]
        L.oc_element_coef.argtypes = [C.c_int, _i64, _ip32, _dp, C.c_double, _dp, _dp]
        L.oc_assemble_elasticity.argtypes = [C.c_int, _i64, _i64, _dp, _ip32, _dp, C.c_double,
                                             C.c_double]
        L.oc_assemble_elasticity.restype = C.c_void_p
        L.oc_assemble_descent.argtypes = [C.c_int, _i64, _i64, _dp, _ip32, _i64, _ip32, _dp,
                                          C.c_double, C.c_double, C.c_double, C.c_int, _dp]
        L.oc_assemble_descent.restype = C.c_void_p
        L.oc_csr_free.argtypes = [C.c_void_p]
        L.oc_csr_rows.argtypes = [C.c_void_p]
        L.oc_csr_rows.restype = _i64
        L.oc_csr_nnz.argtypes = [C.c_void_p]
        L.oc_csr_nnz.restype = _i64
        L.oc_csr_export.argtypes = [C.c_void_p, _ip64, _ip64, _dp]
        L.oc_csr_matvec.argtypes = [C.c_void_p, _dp, _dp]
        L.oc_solve_constrained.argtypes = [C.c_void_p, _up8, _dp, _dp, C.c_double, _i64, _dp,
                                           C.POINTER(C.c_int)]
        L.oc_solve_constrained.restype = _i64
        L.oc_shape_derivative.argtypes = [C.c_int, _i64, _i64, _dp, _ip32, _dp, _dp, C.c_double,
                                          C.c_double, _dp, C.c_int, _i64, C.c_double, C.c_double,
                                          _dp, _dp, _dp, _dp]
        L.oc_shape_derivative.restype = C.c_int
        L.oc_levelset_update.argtypes = [C.c_int, _i64, _i64, _dp, _ip32, _dp, C.c_double, _dp,
                                         _dp]
        L.oc_levelset_update.restype = C.c_int
        L.oc_transport_h2.argtypes = [C.c_int, _i64, _dp, _ip32]
        L.oc_transport_h2.restype = C.c_double
        L.oc_assemble_transport.argtypes = [C.c_int, _i64, _i64, _dp, _ip32, _dp, C.c_double, C.c_int,
                                            C.c_double, C.c_double]
        L.oc_assemble_transport.restype = C.c_void_p
        L.oc_bicgstab.argtypes = [C.c_void_p, _dp, _dp, C.c_double, _i64, _dp, C.POINTER(C.c_int)]
        L.oc_bicgstab.restype = _i64
        L.oc_transport.argtypes = [C.c_int, _i64, _i64, _dp, _ip32, _dp, C.c_double, C.c_int, C.c_double,
                                   C.c_int, C.c_double, _i64, _dp, _dp, C.POINTER(_i64)]
        L.oc_transport.restype = C.c_int
        L.oc_element_geometry.argtypes = [C.c_int, _i64, _dp, _ip32, _dp, _dp]
        L.oc_element_geometry.restype = C.c_int
        L.oc_set_threads.argtypes = [C.c_int]
        L.oc_get_threads.restype = C.c_int
        _lib = L
    return _lib


def _d(a):
    return a.ctypes.data_as(_dp)


def _c64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def _c32(a):
    return np.ascontiguousarray(a, dtype=np.int32)


def set_threads(n: int) -> None:
    lib().oc_set_threads(int(n))


def get_threads() -> int:
    return int(lib().oc_get_threads())


def lame(E: float, nu: float, dim: int, plane_stress: int):
    lam, mu = C.c_double(), C.c_double()
    lib().oc_lame(E, nu, dim, plane_stress, C.byref(lam), C.byref(mu))
    return lam.value, mu.value


def element_coef(dim, conn, phi, ersatz):
    conn = _c32(conn)
    E = conn.shape[1]
    A = np.empty(E)
    chi = np.empty(E)
    lib().oc_element_coef(dim, E, conn.ctypes.data_as(_ip32), _d(_c64(phi)), ersatz, _d(A), _d(chi))
    return A, chi


def element_geometry(dim, coords, conn):
    coords, conn = _c64(coords), _c32(conn)
    E = conn.shape[1]
    vol = np.empty(E)
    grad = np.empty((E, dim + 1, dim))
    rc = lib().oc_element_geometry(dim, E, _d(coords), conn.ctypes.data_as(_ip32), _d(vol),
                                   _d(grad))
    if rc:
        raise ValueError("degenerate element")
    return vol, grad


class CSR:
    """Owning handle of an oracle compressed-row matrix."""

    def __init__(self, handle):
        if not handle:
            raise ValueError("assembly failed (degenerate element)")
        self.h = C.c_void_p(handle)

    def __del__(self):
        if getattr(self, "h", None) and _lib is not None:
            _lib.oc_csr_free(self.h)
            self.h = None

    @property
    def n(self) -> int:
        return int(lib().oc_csr_rows(self.h))

    @property
    def nnz(self) -> int:
        return int(lib().oc_csr_nnz(self.h))

    def matvec(self, x):
        x = _c64(x)
        y = np.empty(self.n)
        lib().oc_csr_matvec(self.h, _d(x), _d(y))
        return y

    def to_scipy(self):
        import scipy.sparse as sp
        n, nnz = self.n, self.nnz
        rp = np.empty(n + 1, dtype=np.int64)
        col = np.empty(nnz, dtype=np.int64)
        val = np.empty(nnz)
        lib().oc_csr_export(self.h, rp.ctypes.data_as(_ip64), col.ctypes.data_as(_ip64), _d(val))
        return sp.csr_matrix((val, col, rp), shape=(n, n))

    def diagonal(self):
        return np.asarray(self.to_scipy().diagonal())

    def solve(self, b, fixed=None, rtol=1e-12, max_iter=1_000_000):
        """Jacobi-PCG from 0 with the clamped unknowns eliminated."""
        b = _c64(b)
        u = np.empty(self.n)
        rr = C.c_double()
        st = C.c_int()
        fx = None if fixed is None else np.ascontiguousarray(fixed, dtype=np.uint8)
        it = lib().oc_solve_constrained(self.h, None if fx is None else fx.ctypes.data_as(_up8),
                                        _d(b), _d(u), rtol, int(max_iter), C.byref(rr),
                                        C.byref(st))
        return u, SolveInfo(int(it), rr.value, st.value)


@dataclass
class SolveInfo:
    iters: int
    relres: float
    status: int


def assemble_elasticity(dim, coords, conn, A_e, lam, mu) -> CSR:
    coords, conn, A_e = _c64(coords), _c32(conn), _c64(A_e)
    N, E = coords.shape[0], conn.shape[1]
    return CSR(lib().oc_assemble_elasticity(dim, N, E, _d(coords), conn.ctypes.data_as(_ip32),
                                            _d(A_e), lam, mu))


def assemble_descent(dim, coords, conn, bfacets, bnormal, alpha, gamma_n, gamma_s, boxes=None) -> CSR:
    coords, conn = _c64(coords), _c32(conn)
    bfacets, bnormal = _c32(bfacets), _c64(bnormal)
    N, E, F = coords.shape[0], conn.shape[1], bfacets.shape[1]
    boxes = np.zeros((0, 2 * dim)) if boxes is None else _c64(boxes).reshape(-1, 2 * dim)
    bx = _c64(boxes)
    return CSR(lib().oc_assemble_descent(dim, N, E, _d(coords), conn.ctypes.data_as(_ip32), F,
                                         bfacets.ctypes.data_as(_ip32), _d(bnormal), alpha,
                                         gamma_n, gamma_s, bx.shape[0],
                                         _d(bx) if bx.size else None))


def shape_derivative(dim, coords, conn, A_e, chi_e, lam, mu, u, lambda_vol=0.0, V=1.0,
                     want_S1=False):
    """Returns (rhs [N*d], S1 [d*d, E] or None, J [n_rhs], vol)."""
    coords, conn = _c64(coords), _c32(conn)
    N, E = coords.shape[0], conn.shape[1]
    U = _c64(u)
    if U.ndim == 1:
        U = U.reshape(-1, 1)
    n_rhs = U.shape[1]
    rhs = np.empty(N * dim)
    S1 = np.empty((dim * dim, E)) if want_S1 else None
    J = np.empty(n_rhs)
    vol = C.c_double()
    rc = lib().oc_shape_derivative(dim, N, E, _d(coords), conn.ctypes.data_as(_ip32), _d(_c64(A_e)),
                                   _d(_c64(chi_e)), lam, mu, _d(U), n_rhs, n_rhs, lambda_vol, V,
                                   _d(rhs), _d(S1) if want_S1 else None, _d(J), C.byref(vol))
    if rc:
        raise ValueError("degenerate element")
    return rhs, S1, J, vol.value


def levelset_update(dim, coords, conn, theta, dt, phi):
    coords, conn = _c64(coords), _c32(conn)
    N, E = coords.shape[0], conn.shape[1]
    out = np.empty(N)
    rc = lib().oc_levelset_update(dim, N, E, _d(coords), conn.ctypes.data_as(_ip32),
                                  _d(_c64(theta)), dt, _d(_c64(phi)), _d(out))
    if rc:
        raise ValueError("degenerate element")
    return out


def transport_h2(dim, coords, conn) -> float:
    """h^2 of the transport diffusion: the paper's mesh-diameter expression
    (Section "Transport equation"), read as h^2."""
    coords, conn = _c64(coords), _c32(conn)
    return float(lib().oc_transport_h2(dim, conn.shape[1], _d(coords), conn.ctypes.data_as(_ip32)))


def assemble_transport(dim, coords, conn, theta, h2, smooth, dt, sign) -> CSR:
    """Step matrix of eq. weak_transport: sign +1 left-hand side L, -1
    right-hand side R (see fo_oracle.c)."""
    coords, conn = _c64(coords), _c32(conn)
    N, E = coords.shape[0], conn.shape[1]
    return CSR(lib().oc_assemble_transport(dim, N, E, _d(coords), conn.ctypes.data_as(_ip32),
                                           _d(_c64(theta)), float(h2), int(bool(smooth)), float(dt),
                                           float(sign)))


def bicgstab(A: CSR, b, x0=None, rtol=1e-12, max_iter=100_000):
    """Jacobi-preconditioned BiCGStab on an oracle matrix from x0 (default 0)."""
    b = _c64(b)
    x = np.zeros(A.n) if x0 is None else _c64(x0).copy()
    rr = C.c_double()
    st = C.c_int()
    it = lib().oc_bicgstab(A.h, _d(b), _d(x), float(rtol), int(max_iter), C.byref(rr), C.byref(st))
    return x, SolveInfo(int(it), rr.value, st.value)


def transport(dim, coords, conn, theta, dt, steps, phi, smooth=True, h2=None, rtol=1e-12,
              max_iter=100_000):
    """`steps` Crank-Nicolson Petrov-Galerkin steps of eq. weak_transport;
    returns (phi_new, operator applications)."""
    coords, conn = _c64(coords), _c32(conn)
    N, E = coords.shape[0], conn.shape[1]
    if h2 is None:
        h2 = transport_h2(dim, coords, conn)
    out = np.empty(N)
    its = _i64()
    rc = lib().oc_transport(dim, N, E, _d(coords), conn.ctypes.data_as(_ip32), _d(_c64(theta)),
                            float(h2), int(bool(smooth)), float(dt), int(steps), float(rtol),
                            int(max_iter), _d(_c64(phi)), _d(out), C.byref(its))
    if rc == -1:
        raise ValueError("degenerate element")
    if rc:
        raise RuntimeError("transport solve did not converge")
    return out, int(its.value)


# ----------------------------------------------------------------------------
# one iteration of the hot path, end to end


@dataclass
class IterationResult:
    u: np.ndarray
    J: np.ndarray
    vol: float
    rhs: np.ndarray
    S1: Optional[np.ndarray]
    theta: np.ndarray
    B_tt: float
    phi_new: Optional[np.ndarray]
    state_info: list
    descent_info: SolveInfo
    A_e: np.ndarray
    chi_e: np.ndarray
    times: dict


def run_iteration(w, rtol=1e-12, lambda_vol=0.0, V=1.0, dt=None, want_S1=False,
                  max_iter=1_000_000) -> IterationResult:
    """State solve(s), shape derivative, descent solve and (if dt is given) the
    level-set update for a fo_inputs.Workload, all in FP64 on the CPU."""
    m = w.mesh
    dim = m.dim
    times = {}
    t0 = time.perf_counter()
    lam, mu = lame(w.E, w.nu, dim, w.plane_stress)
    A_e, chi = element_coef(dim, m.conn, w.phi, w.ersatz)
    K = assemble_elasticity(dim, m.coords, m.conn, A_e, lam, mu)
    times["assemble_state"] = time.perf_counter() - t0
    B = w.b.reshape(m.n_dofs, -1)
    U = np.empty_like(B)
    infos = []
    t0 = time.perf_counter()
    for k in range(B.shape[1]):
        U[:, k], info = K.solve(B[:, k], w.fixed, rtol=rtol, max_iter=max_iter)
        infos.append(info)
    times["state_solve"] = time.perf_counter() - t0
    t0 = time.perf_counter()
    rhs, S1, J, vol = shape_derivative(dim, m.coords, m.conn, A_e, chi, lam, mu, U, lambda_vol,
                                       V, want_S1)
    times["shape_derivative"] = time.perf_counter() - t0
    t0 = time.perf_counter()
    Bd = assemble_descent(dim, m.coords, m.conn, m.bfacets, m.bnormal, w.alpha, w.gamma_n,
                          w.gamma_s, w.boxes)
    times["assemble_descent"] = time.perf_counter() - t0
    t0 = time.perf_counter()
    theta, dinfo = Bd.solve(rhs, None, rtol=rtol, max_iter=max_iter)
    times["descent_solve"] = time.perf_counter() - t0
    B_tt = float(theta @ rhs)
    phi_new = None
    if dt is not None:
        phi_new = levelset_update(dim, m.coords, m.conn, theta, dt, w.phi)
    u_out = U[:, 0] if w.b.ndim == 1 else U
    return IterationResult(u_out, J, vol, rhs, S1, theta, B_tt, phi_new, infos, dinfo, A_e, chi,
                           times)


def adaptive_dt(B_tt, dfactor=1e-2, t_range=(1e-3, 1e-1), s_range=(8, 16)):
    """Final time and step count of the paper's adaptive time stepping
    (Section "Other implementation aspects", eqs. tend and steps), without
    the optional noise: t_end = clip(dfactor / B(theta,theta)),
    s = round((s_max - s_min) ((t_end - t_min)/(t_max - t_min))^(1/6) + s_min);
    returns (t_end, s, dt = t_end / s)."""
    tmin, tmax = t_range
    smin, smax = s_range
    t_end = dfactor / max(B_tt, 1e-300)
    t_end = min(max(t_end, tmin), tmax)
    s = (smax - smin) * ((t_end - tmin) / (tmax - tmin)) ** (1.0 / 6.0) + smin
    s = int(round(min(max(s, smin), smax)))
    return t_end, s, t_end / s
