"""Seeded synthetic inputs shared by the HIP path and the CPU oracle.

This module produces problem data only -- meshes, level sets, load vectors,
clamp masks, boundary facets and seeds.  It contains none of the method's
arithmetic (no stiffness, no solve, no shape derivative, no transport):
those live separately in the oracle and in the HIP library.

Workloads follow the compliance cantilevers of the paper (Section
"Compliance minimization", Examples 1 and 2): a box D, clamped on x = 0,
loaded by a traction patch on the face x = Lx.
"""
from __future__ import annotations

import dataclasses
import functools
import math
from typing import List, Optional, Sequence, Tuple

import numpy as np

# The six axis permutations that define the Kuhn split of a cube.
KUHN_PERMS = ((0, 1, 2), (0, 2, 1), (1, 0, 2), (1, 2, 0), (2, 0, 1), (2, 1, 0))


@dataclasses.dataclass
class Mesh:
    """Conforming simplicial mesh.

    coords : float64 [N, d]   node-blocked coordinates
    conn   : int32 [d+1, E]   element -> node, structure of arrays
    bfacets: int32 [d, F]     boundary facets (nodes of each facet)
    bnormal: float64 [F, d]   unit outward normal of each boundary facet
    """

    dim: int
    coords: np.ndarray
    conn: np.ndarray
    bfacets: np.ndarray
    bnormal: np.ndarray
    lengths: Tuple[float, ...]
    cells: Tuple[int, ...]

    @property
    def n_nodes(self) -> int:
        return int(self.coords.shape[0])

    @property
    def n_elems(self) -> int:
        return int(self.conn.shape[1])

    @property
    def n_dofs(self) -> int:
        return self.n_nodes * self.dim

    @property
    def h(self) -> float:
        return float(self.lengths[0]) / float(self.cells[0])


def _grid_coords(lengths, cells):
    axes = [np.array([L * i / n for i in range(n + 1)], dtype=np.float64)
            for L, n in zip(lengths, cells)]
    grids = np.meshgrid(*axes, indexing="ij")
    # node index = i + (nx+1)*(j + (ny+1)*k): x fastest
    cols = [g.transpose(*reversed(range(len(cells)))).reshape(-1) for g in grids]
    return np.stack(cols, axis=1).copy()


def structured_mesh(cells: Sequence[int], lengths: Sequence[float]) -> Mesh:
    """Structured simplicial mesh of the box prod [0, L_k].

    2D: nx*ny squares, each split along its (i,j)-(i+1,j+1) diagonal.
    3D: nx*ny*nz cubes, each split into the six Kuhn tetrahedra
        {v0, v0+e_p0, v0+e_p0+e_p1, v0+e0+e1+e2} for every permutation p.
    Nodes are numbered lexicographically, x fastest; elements cell by cell.
    """
    cells = tuple(int(c) for c in cells)
    lengths = tuple(float(L) for L in lengths)
    dim = len(cells)
    if dim not in (2, 3) or len(lengths) != dim:
        raise ValueError("dim must be 2 or 3")
    coords = _grid_coords(lengths, cells)
    if dim == 2:
        nx, ny = cells
        sx = 1
        sy = nx + 1
        i, j = np.meshgrid(np.arange(nx), np.arange(ny), indexing="ij")
        v0 = (i + sy * j).T.reshape(-1).astype(np.int64)  # cell order: x fastest
        t1 = np.stack([v0, v0 + sx, v0 + sx + sy])
        t2 = np.stack([v0, v0 + sx + sy, v0 + sy])
        conn = np.empty((3, 2 * v0.size), dtype=np.int64)
        conn[:, 0::2] = t1
        conn[:, 1::2] = t2
    else:
        nx, ny, nz = cells
        step = (1, nx + 1, (nx + 1) * (ny + 1))
        i, j, k = np.meshgrid(np.arange(nx), np.arange(ny), np.arange(nz), indexing="ij")
        v0 = (i + step[1] * j + step[2] * k).transpose(2, 1, 0).reshape(-1).astype(np.int64)
        conn = np.empty((4, 6 * v0.size), dtype=np.int64)
        top = v0 + step[0] + step[1] + step[2]
        for t, p in enumerate(KUHN_PERMS):
            a = v0 + step[p[0]]
            b = a + step[p[1]]
            conn[0, t::6] = v0
            conn[1, t::6] = a
            conn[2, t::6] = b
            conn[3, t::6] = top
    bf, bn = _structured_boundary(cells)
    return Mesh(dim, coords, np.ascontiguousarray(conn.astype(np.int32)),
                np.ascontiguousarray(bf.astype(np.int32)), bn, lengths, cells)


def _structured_boundary(cells):
    """Boundary facets of the structured mesh, with outward unit normals.

    On every box face the simplices restrict to the 2D split of that face
    along the diagonal from its lowest to its highest corner.
    """
    dim = len(cells)
    facets, normals = [], []
    if dim == 2:
        nx, ny = cells
        sy = nx + 1
        for axis, (n_along, stride_along, other_n, stride_other) in enumerate(
                [(ny, sy, nx, 1), (nx, 1, ny, sy)]):
            # axis 0: faces x = 0 / x = Lx (segments along y); axis 1: y faces
            base = np.arange(n_along) * stride_along
            for side, off in ((-1.0, 0), (1.0, other_n * stride_other)):
                f = np.stack([base + off, base + off + stride_along])
                nrm = np.zeros((n_along, 2))
                nrm[:, axis] = side
                facets.append(f)
                normals.append(nrm)
    else:
        nx, ny, nz = cells
        stride = (1, nx + 1, (nx + 1) * (ny + 1))
        for axis in range(3):
            u, v = [a for a in range(3) if a != axis]
            nu, nv = cells[u], cells[v]
            iu, iv = np.meshgrid(np.arange(nu), np.arange(nv), indexing="ij")
            iu = iu.T.reshape(-1)
            iv = iv.T.reshape(-1)
            for side, plane in ((-1.0, 0), (1.0, cells[axis])):
                c0 = plane * stride[axis] + iu * stride[u] + iv * stride[v]
                c_u = c0 + stride[u]
                c_v = c0 + stride[v]
                c_uv = c0 + stride[u] + stride[v]
                f1 = np.stack([c0, c_u, c_uv])
                f2 = np.stack([c0, c_v, c_uv])
                f = np.concatenate([f1, f2], axis=1)
                nrm = np.zeros((f.shape[1], 3))
                nrm[:, axis] = side
                facets.append(f)
                normals.append(nrm)
    return np.concatenate(facets, axis=1), np.ascontiguousarray(np.concatenate(normals, axis=0))


# ----------------------------------------------------------------------------
# level sets (Omega = {phi < 0})


def levelset_cos_holes(coords: np.ndarray) -> np.ndarray:
    """phi(x, y) = -cos(4 pi x) cos(4 pi y) - 0.4  (a periodic array of holes)."""
    x, y = coords[:, 0], coords[:, 1]
    return -np.cos(4 * np.pi * x) * np.cos(4 * np.pi * y) - 0.4


def levelset_balls(coords: np.ndarray, centers: np.ndarray, radii, factor: float = 1.0,
                   ord=2) -> np.ndarray:
    """Initial level set of the paper (Section "Other implementation aspects",
    eq. (phi0)): phi = factor * max_k (r_k - |x - c_k|_ord).

    factor > 0 makes Omega the box with ball-shaped holes; factor < 0 makes it
    the union of the balls.
    """
    centers = np.atleast_2d(np.asarray(centers, dtype=np.float64))
    radii = np.broadcast_to(np.asarray(radii, dtype=np.float64), (centers.shape[0],))
    best = np.full(coords.shape[0], -np.inf)
    for c, r in zip(centers, radii):
        d = np.linalg.norm(coords - c[None, :], ord=ord, axis=1)
        np.maximum(best, r - d, out=best)
    return factor * best


def lattice_centers(counts: Sequence[int], lengths: Sequence[float]) -> np.ndarray:
    """Centres of the cells of a counts[0] x counts[1] (x counts[2]) lattice on the box."""
    axes = [np.array([(i + 0.5) * L / n for i in range(n)]) for n, L in zip(counts, lengths)]
    g = np.meshgrid(*axes, indexing="ij")
    return np.stack([a.reshape(-1) for a in g], axis=1)


# ----------------------------------------------------------------------------
# loads, clamps, penalised subdomains


def clamp_mask(mesh: Mesh, axis: int = 0, value: float = 0.0) -> np.ndarray:
    """uint8 [N*d]: all components of nodes on the plane x_axis == value are fixed."""
    on = mesh.coords[:, axis] == value
    m = np.repeat(on, mesh.dim).astype(np.uint8)
    return m


def _clip_polygon(poly: List[Tuple[float, float]], lo, hi):
    """Sutherland-Hodgman clip of a convex polygon against [lo0,hi0] x [lo1,hi1]."""
    def clip(pts, axis, bound, keep_ge):
        out = []
        n = len(pts)
        for idx in range(n):
            p, q = pts[idx], pts[(idx + 1) % n]
            ip = (p[axis] >= bound) if keep_ge else (p[axis] <= bound)
            iq = (q[axis] >= bound) if keep_ge else (q[axis] <= bound)
            if ip:
                out.append(p)
            if ip != iq:
                t = (bound - p[axis]) / (q[axis] - p[axis])
                out.append((p[0] + t * (q[0] - p[0]), p[1] + t * (q[1] - p[1])))
        return out
    for axis in range(2):
        if not poly:
            return poly
        poly = clip(poly, axis, lo[axis], True)
        if not poly:
            return poly
        poly = clip(poly, axis, hi[axis], False)
    return poly


def _polygon_area_centroid(poly):
    a = 0.0
    cx = cy = 0.0
    n = len(poly)
    for idx in range(n):
        x0, y0 = poly[idx]
        x1, y1 = poly[(idx + 1) % n]
        cr = x0 * y1 - x1 * y0
        a += cr
        cx += (x0 + x1) * cr
        cy += (y0 + y1) * cr
    a *= 0.5
    if abs(a) < 1e-300:
        return 0.0, (0.0, 0.0)
    return abs(a), (cx / (6 * a), cy / (6 * a))


def traction_load(mesh: Mesh, traction: Sequence[float], lo: Sequence[float],
                  hi: Sequence[float], axis: int = 0, side: float = 1.0) -> np.ndarray:
    """Load vector b[a*d + i] = t_i * integral over the patch of the hat function N_a.

    The patch is the part of the face x_axis = (side>0 ? L_axis : 0) whose
    in-face coordinates lie in [lo, hi] (one interval in 2D, a rectangle in
    3D).  Facets are clipped to the patch exactly; since N_a is affine on a
    facet its integral over the clipped piece is |piece| * N_a(centroid).
    """
    d = mesh.dim
    t = np.asarray(traction, dtype=np.float64)
    b = np.zeros(mesh.n_nodes * d)
    sel = mesh.bnormal[:, axis] == side
    facets = mesh.bfacets[:, sel]
    others = [a for a in range(d) if a != axis]
    X = mesh.coords
    if d == 2:
        o = others[0]
        for f in facets.T:
            ya, yb = X[f[0], o], X[f[1], o]
            lo_f, hi_f = min(ya, yb), max(ya, yb)
            s0, s1 = max(lo_f, lo[0]), min(hi_f, hi[0])
            if s1 <= s0:
                continue
            mid = 0.5 * (s0 + s1)
            L = s1 - s0
            n0 = (yb - mid) / (yb - ya)
            for node, w in ((f[0], n0), (f[1], 1.0 - n0)):
                b[node * d:node * d + d] += t * L * w
    else:
        for f in facets.T:
            P = X[f][:, others]  # 3 x 2 in-face coordinates
            poly = _clip_polygon([tuple(p) for p in P], lo, hi)
            if len(poly) < 3:
                continue
            area, c = _polygon_area_centroid(poly)
            if area <= 0.0:
                continue
            # barycentric coordinates of the centroid in the facet triangle
            T = np.array([[P[1, 0] - P[0, 0], P[2, 0] - P[0, 0]],
                          [P[1, 1] - P[0, 1], P[2, 1] - P[0, 1]]])
            l12 = np.linalg.solve(T, np.array([c[0] - P[0, 0], c[1] - P[0, 1]]))
            w = (1.0 - l12[0] - l12[1], l12[0], l12[1])
            for node, wk in zip(f, w):
                b[node * d:node * d + d] += t * area * wk
    return b


def patch_area(lo, hi) -> float:
    return float(np.prod(np.asarray(hi, dtype=np.float64) - np.asarray(lo, dtype=np.float64)))


# ----------------------------------------------------------------------------
# configured workloads


@dataclasses.dataclass
class Workload:
    """Everything one iteration of the hot path needs, all on the host."""

    name: str
    mesh: Mesh
    phi: np.ndarray              # float64 [N]
    b: np.ndarray                # float64 [N*d] or [N*d, n_rhs] (RHS contiguous)
    fixed: np.ndarray            # uint8 [N*d]
    E: float = 1.0
    nu: float = 0.3
    plane_stress: int = 1
    ersatz: float = 1e-3
    alpha: float = 0.01          # descent: mass weight
    gamma_n: float = 1e4         # descent: boundary normal penalty
    gamma_s: float = 1e4         # descent: penalised subdomain weight
    boxes: Optional[np.ndarray] = None   # [n_boxes, 2*d] (lo..., hi...) open boxes
    patch_lo: Tuple[float, ...] = ()
    patch_hi: Tuple[float, ...] = ()

    @property
    def n_rhs(self) -> int:
        return 1 if self.b.ndim == 1 else int(self.b.shape[1])


def omega0_boxes(dim: int) -> np.ndarray:
    """Penalised subdomain around the load (Compliance Examples 1 and 2)."""
    if dim == 2:
        return np.array([[1.95, 0.42, 2.0 + 1e-9, 0.58]])
    return np.array([[1.90, 0.35, 0.35, 2.0 + 1e-9, 0.65, 0.65]])


def sphere_hole_centers_4x2x2() -> np.ndarray:
    return lattice_centers((4, 2, 2), (2.0, 1.0, 1.0))


def cantilever_2d(cells=(64, 32)) -> Workload:
    """2D plane-stress cantilever on [0,2]x[0,1]: cosine holes, clamp x=0,
    unit downward traction on {2} x [0.45, 0.55]."""
    mesh = structured_mesh(cells, (2.0, 1.0))
    phi = levelset_cos_holes(mesh.coords)
    lo, hi = (0.45,), (0.55,)
    b = traction_load(mesh, (0.0, -1.0), lo, hi)
    return Workload("cantilever2d_%dx%d" % cells, mesh, phi, b, clamp_mask(mesh),
                    boxes=omega0_boxes(2), patch_lo=lo, patch_hi=hi)


def cantilever_3d(cells=(96, 48, 48), holes: bool = True) -> Workload:
    """3D cantilever on [0,2]x[0,1]^2: 16 spherical holes of radius 0.15 at the
    4x2x2 lattice centres, clamp x=0, unit -z traction on a 0.1x0.1 patch at
    the centre of the face x=2."""
    mesh = structured_mesh(cells, (2.0, 1.0, 1.0))
    phi = levelset_balls(mesh.coords, sphere_hole_centers_4x2x2(), 0.15,
                         factor=1.0 if holes else -1.0)
    lo, hi = (0.45, 0.45), (0.55, 0.55)
    b = traction_load(mesh, (0.0, 0.0, -1.0), lo, hi)
    return Workload("cantilever3d_%dx%dx%d" % cells, mesh, phi, b, clamp_mask(mesh),
                    plane_stress=0, boxes=omega0_boxes(3), patch_lo=lo, patch_hi=hi)


def multi_load_3d(cells=(64, 32, 32), n_loads: int = 64, seed: int = 3) -> Workload:
    """Batched load cases on one level set: patch 0.1x0.1 on the face x=2 with
    centre uniform on [0.05,0.95]^2, unit direction uniform on the sphere."""
    w = cantilever_3d(cells)
    rng = np.random.default_rng(seed)
    centers = rng.uniform(0.05, 0.95, size=(n_loads, 2))
    dirs = rng.standard_normal((n_loads, 3))
    dirs /= np.linalg.norm(dirs, axis=1, keepdims=True)
    B = np.zeros((w.mesh.n_dofs, n_loads))
    for k in range(n_loads):
        lo = tuple(centers[k] - 0.05)
        hi = tuple(centers[k] + 0.05)
        B[:, k] = traction_load(w.mesh, dirs[k], lo, hi)
    w.b = np.ascontiguousarray(B)
    w.name = "multiload3d_%dx%dx%d_s%d" % (cells + (n_loads,))
    return w


def multi_load_2d(cells=(64, 32), n_loads: int = 16, seed: int = 5) -> Workload:
    """2D counterpart of multi_load_3d: load segments of length 0.1 on the face
    x=2 with centre uniform on [0.05,0.95], unit direction uniform on the circle."""
    w = cantilever_2d(cells)
    rng = np.random.default_rng(seed)
    centers = rng.uniform(0.05, 0.95, size=n_loads)
    ang = rng.uniform(0.0, 2.0 * np.pi, size=n_loads)
    B = np.zeros((w.mesh.n_dofs, n_loads))
    for k in range(n_loads):
        B[:, k] = traction_load(w.mesh, (np.cos(ang[k]), np.sin(ang[k])), (centers[k] - 0.05,),
                                (centers[k] + 0.05,))
    w.b = np.ascontiguousarray(B)
    w.name = "multiload2d_%dx%d_s%d" % (cells + (n_loads,))
    return w


SERVING_MESHES = (("2d", (128, 64)), ("2d", (256, 128)), ("3d", (32, 16, 16)),
                  ("3d", (64, 32, 32)), ("3d", (80, 40, 40)))


class InverseWorkload:
    """Inverse elasticity (Kohn-Vogelius) inputs, all on the host: the mesh
    with its boundary facets restricted to Gamma_1 (the faces other than
    x = 0), the clamp masks of Gamma_0 and of the whole boundary, one force
    f on Gamma_1 with its displacement data g (a field on the whole domain
    that vanishes on Gamma_0, here linear: g(x) = x_0 a), the initial level
    set (a disk or ball of the stiffer material) and the weights."""

    def __init__(self, mesh, fixed0, fixed_all, f, g, phi, kappa=10.0, alpha=1.0, beta=1.0, E=1.0, nu=0.3,
                 plane_stress=1, fs=None, gs=None):
        self.mesh, self.fixed0, self.fixed_all = mesh, fixed0, fixed_all
        self.f, self.g, self.phi = f, g, phi
        self.kappa, self.alpha, self.beta = kappa, alpha, beta
        self.E, self.nu, self.plane_stress = E, nu, plane_stress
        # all pairs (f_k, g_k); pair 0 is (f, g)
        self.fs = [f] if fs is None else list(fs)
        self.gs = [g] if gs is None else list(gs)

    @property
    def n_pairs(self) -> int:
        return len(self.fs)

    def pair(self, k: int) -> "InverseWorkload":
        """The single-pair workload of pair k."""
        return InverseWorkload(self.mesh, self.fixed0, self.fixed_all, self.fs[k], self.gs[k], self.phi, self.kappa,
                               self.alpha, self.beta, self.E, self.nu, self.plane_stress)

    def columns(self, arrays) -> np.ndarray:
        """The pairs' vectors as the columns of an [n_dofs][n_pairs] array."""
        return np.ascontiguousarray(np.stack(arrays, axis=1))


def inverse_elasticity(cells, g_scale=(0.02, -0.01, 0.015), n_pairs: int = 1) -> InverseWorkload:
    """[0,2]x[0,1] (2D) or [0,2]x[0,1]^2 (3D); Gamma_0 = {x = 0}; an inward
    unit traction on the middle of the face x = 2; an inclusion of radius
    0.25 centred at (1, 0.5[, 0.5]).  With n_pairs > 1, pair k >= 1 tilts
    the traction by 0.35 k radians towards +y and moves its patch (width 0.4)
    to y centred at 0.5 + 0.25 sin(1.3 k); its data g_k = x_0 a_k with a_k =
    (a_0 cos 0.7k, a_1 + 0.004 k, a_2 sin(0.7k + 1))."""
    d = len(cells)
    lengths = (2.0, 1.0) if d == 2 else (2.0, 1.0, 1.0)
    base = structured_mesh(cells, lengths)
    keep = base.bnormal[:, 0] != -1.0
    mesh = Mesh(base.dim, base.coords, base.conn, np.ascontiguousarray(base.bfacets[:, keep]),
                np.ascontiguousarray(base.bnormal[keep]), base.lengths, base.cells)
    lo, hi = ((0.3,), (0.7,)) if d == 2 else ((0.3, 0.3), (0.7, 0.7))
    f = traction_load(base, (-1.0,) + (0.0,) * (d - 1), lo, hi)
    bnodes = np.unique(base.bfacets.ravel())
    fixed_all = np.zeros(mesh.n_nodes * d, dtype=np.uint8)
    for i in range(d):
        fixed_all[bnodes * d + i] = 1
    a = np.asarray(g_scale[:d], dtype=np.float64)
    g = (mesh.coords[:, :1] * a[None, :]).ravel()
    c = np.array([1.0, 0.5, 0.5][:d])
    phi = np.linalg.norm(mesh.coords - c, axis=1) - 0.25
    fs, gs = [f], [g]
    for k in range(1, n_pairs):
        t = 0.35 * k
        direction = (-np.cos(t), np.sin(t)) + ((0.5 * np.sin(t),) if d == 3 else ())
        yc = 0.5 + 0.25 * np.sin(1.3 * k)
        lo_k = (yc - 0.2,) if d == 2 else (yc - 0.2, 0.3)
        hi_k = (yc + 0.2,) if d == 2 else (yc + 0.2, 0.7)
        fs.append(traction_load(base, direction, lo_k, hi_k))
        ak = np.array([g_scale[0] * np.cos(0.7 * k), g_scale[1] + 0.004 * k, g_scale[2] * np.sin(0.7 * k + 1.0)])
        gs.append((mesh.coords[:, :1] * ak[None, :d]).ravel())
    return InverseWorkload(mesh, clamp_mask(base), fixed_all, f, g, phi, plane_stress=1 if d == 2 else 0,
                           fs=fs, gs=gs)


@functools.lru_cache(maxsize=8)
def _shared_mesh(cells, lengths) -> Mesh:
    """Structured mesh shared (read-only) by the requests on the same grid."""
    return structured_mesh(cells, lengths)


def serving_request(req_id: int, base_seed: int = 1000, meshes=SERVING_MESHES) -> Workload:
    """One serving request: mesh drawn uniformly from `meshes`, 4..16 spherical
    holes of radius 0.15 with uniform centres, a load patch of side 0.1 on the
    face x=2 with uniform centre, unit direction uniform on the circle/sphere."""
    rng = np.random.default_rng(base_seed + req_id)
    kind, cells = meshes[int(rng.integers(len(meshes)))]
    dim = 2 if kind == "2d" else 3
    lengths = (2.0, 1.0) if dim == 2 else (2.0, 1.0, 1.0)
    mesh = _shared_mesh(tuple(cells), lengths)
    n_holes = int(rng.integers(4, 17))
    centers = rng.uniform(0.0, 1.0, size=(n_holes, dim)) * np.asarray(lengths)
    phi = levelset_balls(mesh.coords, centers, 0.15)
    c = rng.uniform(0.05, 0.95, size=dim - 1)
    v = rng.standard_normal(dim)
    v /= np.linalg.norm(v)
    lo, hi = tuple(c - 0.05), tuple(c + 0.05)
    b = traction_load(mesh, v, lo, hi)
    name = "req%d_%s_%s" % (req_id, kind, "x".join(map(str, cells)))
    return Workload(name, mesh, phi, b, clamp_mask(mesh), plane_stress=1 if dim == 2 else 0,
                    boxes=omega0_boxes(dim), patch_lo=lo, patch_hi=hi)


def poisson_arrivals(n: int, rate_per_s: float = 200.0, seed: int = 4) -> np.ndarray:
    """Arrival times (s) of a Poisson stream: exponential gaps of mean 1/rate."""
    rng = np.random.default_rng(seed)
    return np.cumsum(rng.exponential(1.0 / rate_per_s, size=n))


def random_levelset_perturbation(coords: np.ndarray, seed: int, amp: float = 0.05) -> np.ndarray:
    """A smooth seeded field (sum of a few low sine modes) for varying phi."""
    rng = np.random.default_rng(seed)
    out = np.zeros(coords.shape[0])
    for _ in range(4):
        k = rng.integers(1, 4, size=coords.shape[1])
        ph = rng.uniform(0, 2 * math.pi, size=coords.shape[1])
        term = np.ones(coords.shape[0])
        for a in range(coords.shape[1]):
            term *= np.sin(math.pi * k[a] * coords[:, a] + ph[a])
        out += amp * term
    return out
