"""Serving: a stream of hot-path requests through the libfo pool.

A request is one iteration's finite-element work on its own mesh (level set,
state solve, compliance and shape derivative, descent solve).  The pool
(fo_pool_*) admits requests into slots while its device-memory budget has
room and runs each on its own stream, as a fiber on the thread that drives
the pool (fo_pool_wait / fo_pool_step), so that requests admitted while
others run overlap on the GPU; finished contexts stay resident for later
requests on the same mesh.  This module only marshals
requests and drives arrivals in real time; every step runs in libfo.
"""
from __future__ import annotations

import collections
import ctypes as C
import time
from dataclasses import dataclass, field
from typing import List, Optional, Sequence

import numpy as np

from . import fo


def mesh_key(w) -> int:
    """Identity of a workload's mesh and material for context reuse: requests
    with equal keys share resident contexts."""
    m = w.mesh
    h = hash((m.dim, m.n_nodes, m.n_elems, tuple(np.round(m.lengths, 12)), tuple(m.cells),
              w.E, w.nu, w.plane_stress, w.ersatz, w.fixed.tobytes()))
    return (h & 0xFFFFFFFFFFFFFFFF) or 1


@dataclass
class Request:
    """One request: a workload plus host output arrays (kept alive here)."""
    w: object
    key: int = 0
    state_opts: fo.SolveOpts = field(default_factory=lambda: fo.SolveOpts(precision=fo.FO_FP32_IR, rtol=1e-8))
    descent_opts: fo.SolveOpts = field(default_factory=lambda: fo.SolveOpts(rtol=1e-8))
    lambda_vol: float = 0.0
    V: float = 1.0

    def __post_init__(self):
        w = self.w
        m = w.mesh
        n = m.n_dofs
        self._coords = np.ascontiguousarray(m.coords, dtype=np.float64)
        self._conn = np.ascontiguousarray(m.conn, dtype=np.int32)
        self._fixed = np.ascontiguousarray(w.fixed, dtype=np.uint8)
        self._bf = np.ascontiguousarray(m.bfacets, dtype=np.int32)
        self._bn = np.ascontiguousarray(m.bnormal, dtype=np.float64)
        self._phi = np.ascontiguousarray(w.phi, dtype=np.float64)
        self._b = np.ascontiguousarray(np.asarray(w.b).reshape(n), dtype=np.float64)
        self.dopts = fo.DescentOpts(w.alpha, w.gamma_n, w.gamma_s, w.boxes, dim=m.dim)
        self.u = np.zeros(n)
        self.rhs = np.zeros(n)
        self.theta = np.zeros(n)

    def c(self) -> fo.fo_request:
        m = self.w.mesh
        mesh = fo.fo_mesh(m.dim, m.n_nodes, m.n_elems, self._coords.ctypes.data, self._conn.ctypes.data,
                          self._fixed.ctypes.data, int(self._bf.shape[1]), self._bf.ctypes.data,
                          self._bn.ctypes.data)
        mat = fo.fo_material(self.w.E, self.w.nu, int(self.w.plane_stress), self.w.ersatz)
        return fo.fo_request(mesh, mat, self.key, self._phi.ctypes.data, self._b.ctypes.data,
                             self.state_opts.c(), self.descent_opts.c(), self.dopts.c(),
                             self.lambda_vol, self.V, self.u.ctypes.data, self.rhs.ctypes.data,
                             self.theta.ctypes.data)


@dataclass
class Result:
    status: int
    reused_context: bool
    state: fo.Stats
    descent: fo.Stats
    J: float
    vol: float
    B_tt: float
    t_admit: float
    t_start: float
    t_end: float


def _stats(s: fo.fo_solve_stats) -> fo.Stats:
    return fo.Stats(s.status, s.iters_inner, s.iters_outer, s.rel_res, s.seconds)


class Pool:
    """fo_pool_* wrapper.  Times in results are seconds since creation."""

    def __init__(self, budget_bytes: int, max_slots: int = 8):
        h = C.c_void_p()
        fo._check(fo.lib().fo_pool_create(C.byref(h), int(budget_bytes), int(max_slots)), "fo_pool_create")
        self.h = h
        self.t0 = time.perf_counter()
        self._live = {}

    def admit(self, req: Request) -> Optional[int]:
        """Slot of the started request, or None when the pool is busy."""
        slot = C.c_int32(-1)
        q = req.c()
        rc = fo.lib().fo_pool_admit(self.h, C.byref(q), C.byref(slot))
        if rc == fo.FO_ERR_BUSY:
            return None
        fo._check(rc, "fo_pool_admit")
        self._live[slot.value] = (req, q)
        return slot.value

    def step(self) -> int:
        """One scheduling round; returns the number of requests still running."""
        running = C.c_int32(0)
        fo._check(fo.lib().fo_pool_step(self.h, C.byref(running)), "fo_pool_step")
        return running.value

    def wait(self, timeout_s: Optional[float]) -> int:
        slot = C.c_int32(-1)
        us = -1 if timeout_s is None else int(max(timeout_s, 0.0) * 1e6)
        fo._check(fo.lib().fo_pool_wait(self.h, us, C.byref(slot)), "fo_pool_wait")
        return slot.value

    def poll(self, slot: int) -> Optional[Result]:
        done = C.c_int32(0)
        r = fo.fo_pool_result()
        fo._check(fo.lib().fo_pool_poll(self.h, slot, C.byref(done), C.byref(r)), "fo_pool_poll")
        if not done.value:
            return None
        return Result(r.status, bool(r.reused_context), _stats(r.state), _stats(r.descent), r.J, r.vol,
                      r.B_tt, r.t_admit, r.t_start, r.t_end)

    def release(self, slot: int):
        fo._check(fo.lib().fo_pool_release(self.h, slot), "fo_pool_release")
        self._live.pop(slot, None)

    def stats(self) -> dict:
        used, run, res = C.c_size_t(), C.c_int32(), C.c_int32()
        fo._check(fo.lib().fo_pool_stats(self.h, C.byref(used), C.byref(run), C.byref(res)), "fo_pool_stats")
        return {"used_bytes": used.value, "running": run.value, "resident": res.value}

    def close(self):
        if getattr(self, "h", None):
            fo.lib().fo_pool_destroy(self.h)
            self.h = None
            self._live.clear()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def percentile(x: Sequence[float], q: float) -> float:
    """q-th percentile (0..100) by linear interpolation between order statistics."""
    a = np.sort(np.asarray(x, dtype=np.float64))
    if a.size == 0:
        return float("nan")
    pos = (a.size - 1) * q / 100.0
    lo = int(np.floor(pos))
    hi = min(lo + 1, a.size - 1)
    return float(a[lo] + (a[hi] - a[lo]) * (pos - lo))


def serve(requests: List[Request], arrivals: Sequence[float], budget_bytes: int, max_slots: int = 8,
          log=None) -> dict:
    """Replays `requests` arriving at times `arrivals` (seconds, increasing)
    in real time through a pool: FIFO admission as slots and budget free up,
    completion latency = end of the request's work - its arrival."""
    pool = Pool(budget_bytes, max_slots)
    queue = collections.deque()
    n = len(requests)
    done = [None] * n
    slot_of = {}
    nxt = 0
    t_start = time.perf_counter()
    offset = t_start - pool.t0          # pool clock -> arrival clock
    completed = 0
    max_queue = 0
    while completed < n:
        now = time.perf_counter() - t_start
        while nxt < n and arrivals[nxt] <= now:
            queue.append(nxt)
            nxt += 1
        max_queue = max(max_queue, len(queue))
        while queue:
            i = queue[0]
            s = pool.admit(requests[i])
            if s is None:
                break
            queue.popleft()
            slot_of[s] = i
        timeout = 0.002 if nxt >= n else max(0.0, min(0.002, arrivals[nxt] - (time.perf_counter() - t_start)))
        if pool.wait(timeout) >= 0:
            for s in list(slot_of):
                r = pool.poll(s)
                if r is None:
                    continue
                done[slot_of.pop(s)] = r
                pool.release(s)
                completed += 1
    wall = time.perf_counter() - t_start
    pool.close()
    lat = [done[i].t_end - offset - arrivals[i] for i in range(n)]
    service = [done[i].t_end - done[i].t_start for i in range(n)]
    return {
        "requests": n,
        "wall_s": wall,
        "solves_per_s": n / wall,
        "latency_p50_s": percentile(lat, 50),
        "latency_p99_s": percentile(lat, 99),
        "service_p50_s": percentile(service, 50),
        "max_queue": max_queue,
        "reused_contexts": int(sum(1 for r in done if r.reused_context)),
        "statuses": sorted(set(int(r.status) for r in done)),
        "results": done,
        "latencies": lat,
    }
