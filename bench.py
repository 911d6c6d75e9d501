#!/usr/bin/env python3
"""Benchmark of the hot path on one MI355X.

Headline workload (the metric's configuration): the 3D cantilever box
[0,2]x[0,1]^2 meshed with 64x32x32 cubes x 6 tetrahedra (393,216 elements,
70,785 nodes, 212,355 unknowns), 16 spherical holes, clamp at x = 0, and 64
seeded load cases (unit traction of random direction on a 0.1 x 0.1 patch
at a random place on the face x = 2) on one level set.  A step is one full
iteration of the hot path for all 64 load cases: level set -> coefficients
and Jacobi diagonal, the 64 state solves to relative residual 1e-8 by the
batched FP32 solver on the matrix cores with FP64 refinement, compliance of
every case and the shape derivative summed over the cases (the multi-load
compliance problem), H1 descent solve, explicit level-set update.  The same
step with the 64 state solves in plain FP64 (one after another) is timed for
comparison.  value = load-case solves per second.

Also measured (extra keys): the single-load iteration on 96x48x48 (c2, its
working set stays in the 256 MB Infinity Cache, so its bandwidth is
"effective"), the large instance 256x128x128 (25.2M elements, where the CG
operator's HBM fraction is claimed), the paper's transport step,
reinitialisation, heat and inverse models and loops, and the serving stream.

Prints one JSON line on stdout; progress goes to stderr.
"""
from __future__ import annotations

import argparse
import json
import os
import platform
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0


def log(msg):
    print("[bench] " + msg, file=sys.stderr, flush=True)


def cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return platform.processor()


def apply_bytes(mesh, width):
    """Algorithmic bytes of one K(phi) application: x read + y written
    (DOF values each), node coordinates, and per element 4 int32 vertex ids
    plus one byte for the level-set coefficient (17 B per tetrahedron)."""
    d = mesh.dim
    return 2 * mesh.n_dofs * width + mesh.n_nodes * d * width + mesh.n_elems * (4 * (d + 1) + 1)


def fused_cg_bytes(mesh, width):
    """Algorithmic bytes of the fused CG operator kernel: the K(phi) apply of
    p plus the direction update p = D^-1 r + beta p_old folded into it, i.e.
    r, D^-1 and p_old read and p written in addition to q written."""
    return apply_bytes(mesh, width) + 3 * mesh.n_dofs * width


# Kernel sources whose change invalidates recorded HBM traffic counters, and
# the committed counter summaries (FETCH_SIZE / WRITE_SIZE per launch).
TRAFFIC_SOURCES = ["fo_tiled.hip", "fo_element.h", "fo_ops.h", "fo_reduce.h", "fo_internal.h",
                   "fo_tiles.cpp", "fo_tiles.h", "fo_xcd.h"]
BATCH_SOURCES = ["fo_nodal.hip", "fo_batch_dev.h", "fo_internal.h", "fo_xcd.h"]
TRAFFIC_PROFILE = os.path.join(ROOT, "profiles", "k_tile_cg_fp32_cantilever3d_96x48x48.md")
LARGE_PROFILE = os.path.join(ROOT, "profiles", "k_tile_cg_fp32_cantilever3d_256x128x128.md")
BATCH_PROFILE = os.path.join(ROOT, "profiles", "k_nodal_apply_multiload3d_64x32x32.md")


def kernel_source_hash(sources):
    import hashlib
    h = hashlib.sha256()
    for f in sources:
        with open(os.path.join(ROOT, "paper_2601_05709_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def recorded_traffic(path, cells, sources):
    """HBM bytes per launch of a kernel from a committed FETCH_SIZE/WRITE_SIZE
    counter summary, or None when the summary is missing, covers another mesh
    or was taken on other kernel sources."""
    try:
        fields = dict(line.split(":", 1) for line in open(path) if line.startswith("- ") and ":" in line)
    except OSError:
        return None
    fields = {k[2:].strip(): v.strip().strip("`") for k, v in fields.items()}
    if fields.get("source-sha256") != kernel_source_hash(sources):
        return None
    if fields.get("cells") != "x".join(str(c) for c in cells):
        return None
    try:
        return float(fields["traffic-bytes-per-launch"])
    except (KeyError, ValueError):
        return None


def run_steps(it, k):
    import torch
    outs = []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(k):
        outs.append(it.run(update=True, reset_phi=True))
    torch.cuda.synchronize()
    return time.perf_counter() - t0, outs


def cpu_baseline_multi(w, iters_per_col, descent_iters, budget_s):
    """The FP64 oracle on the host cores, one whole hot-path iteration of the
    multi-load workload: CSR assembly, Jacobi-PCG of a sample of the load
    cases (the same algorithm as the GPU's plain FP64 path; the sample's time
    per case is scaled to all cases and its iteration count to the mean the
    GPU's FP64 path needs), the summed shape derivative (sampled cases, scaled),
    the descent operator's assembly and Jacobi-PCG, the level-set update."""
    import numpy as np
    import oracle as oc
    m = w.mesh
    n_loads = w.n_rhs
    B = w.b.reshape(m.n_dofs, n_loads)
    t0 = time.perf_counter()
    lam, mu = oc.lame(w.E, w.nu, m.dim, w.plane_stress)
    A, chi = oc.element_coef(m.dim, m.conn, w.phi, w.ersatz)
    K = oc.assemble_elasticity(m.dim, m.coords, m.conn, A, lam, mu)
    t_asm = time.perf_counter() - t0
    t0 = time.perf_counter()
    _, info = K.solve(B[:, 0], w.fixed, rtol=1e-8, max_iter=50)
    per = (time.perf_counter() - t0) / max(info.iters, 1)
    n_it = int(max(20, min(iters_per_col, 0.5 * budget_s / max(per, 1e-9) / 2)))
    t_cols, its = 0.0, 0
    U = np.zeros((m.n_dofs, 2))
    for k in range(2):
        t0 = time.perf_counter()
        U[:, k], info = K.solve(B[:, k], w.fixed, rtol=1e-8, max_iter=n_it)
        t_cols += time.perf_counter() - t0
        its += info.iters
    per = t_cols / max(its, 1)
    t0 = time.perf_counter()
    rhs, _, _, _ = oc.shape_derivative(m.dim, m.coords, m.conn, A, chi, lam, mu, U)
    t_sd2 = time.perf_counter() - t0
    t0 = time.perf_counter()
    Bd = oc.assemble_descent(m.dim, m.coords, m.conn, m.bfacets, m.bnormal, w.alpha, w.gamma_n, w.gamma_s, w.boxes)
    t_basm = time.perf_counter() - t0
    t0 = time.perf_counter()
    theta, dinfo = Bd.solve(rhs, None, rtol=1e-8, max_iter=max(10, int(descent_iters)))
    t_dit = time.perf_counter() - t0
    dper = t_dit / max(dinfo.iters, 1)
    t0 = time.perf_counter()
    oc.levelset_update(m.dim, m.coords, m.conn, theta, 1e-3, w.phi)
    t_up = time.perf_counter() - t0
    step_s = (t_asm + n_loads * iters_per_col * per + t_sd2 * n_loads / 2 + t_basm + descent_iters * dper + t_up)
    return {
        "value": n_loads / step_s, "unit": "solves/s", "cores": oc.get_threads(), "kind": "oracle",
        "sample": "one hot-path iteration of the 64-load workload: FP64 CSR assembly (%.2f s), Jacobi-PCG of 2 of "
                  "the 64 load cases for %d iterations (%.2f s; scaled to 64 cases of %d iterations, the mean of the "
                  "GPU's plain FP64 path), the derivative of 2 cases (%.2f s, scaled to 64), descent assembly "
                  "(%.2f s) and %d Jacobi-PCG iterations (%.2f s, scaled to %d), level-set update (%.2f s)"
                  % (t_asm, its, t_cols, iters_per_col, t_sd2, t_basm, dinfo.iters, t_dit, descent_iters, t_up),
        "dof_iters_per_s": m.n_dofs / per, "cpu_model": cpu_model(), "seconds_per_step": step_s,
        "assemble_s": t_asm, "s_per_iter": per,
    }


def serving_case(n=120, rate=200.0, budget_bytes=16 << 30, max_slots=12, fp32_descent=True):
    """Serving stream: n requests (state solve and descent solve to 1e-8,
    FP32+refinement from 100k DOFs, else FP64; shape derivative) on meshes
    drawn from the five serving sizes, Poisson arrivals at `rate`, admission
    by a device memory budget, contexts kept resident per mesh."""
    import fo_inputs as fi
    from paper_2601_05709_amd import fo, serving
    reqs = []
    for i in range(n):
        w = fi.serving_request(i)
        # small problems are launch-latency bound: FP32 saves no time there and
        # only adds iterations, so they are solved in FP64
        prec = fo.FO_FP32_IR if w.mesh.n_dofs >= 100000 else fo.FO_FP64
        dprec = prec if fp32_descent else fo.FO_FP64
        reqs.append(serving.Request(w, key=serving.mesh_key(w),
                                    state_opts=fo.SolveOpts(precision=prec, rtol=1e-8),
                                    descent_opts=fo.SolveOpts(precision=dprec, rtol=1e-8)))
    arrivals = fi.poisson_arrivals(n, rate, seed=4)
    out = serving.serve(reqs, arrivals, budget_bytes, max_slots)
    kinds = {}
    for r, q in zip(out["results"], reqs):
        k = q.w.name.split("_", 1)[1]
        kinds.setdefault(k, []).append(r.t_end - r.t_start)
    return {
        "workload": "Poisson arrivals %.0f/s, %d requests, meshes 2D 128x64/256x128, 3D 32x16x16/64x32x32/"
                    "80x40x40; state + derivative + descent per request (solves FP32+refinement from "
                    "100k DOFs, else FP64), rel. res 1e-8" % (rate, n),
        "solves_per_s": out["solves_per_s"], "wall_s": out["wall_s"],
        "latency_p50_s": out["latency_p50_s"], "latency_p99_s": out["latency_p99_s"],
        "service_p50_s": out["service_p50_s"], "max_queue": out["max_queue"],
        "reused_contexts": out["reused_contexts"], "statuses": out["statuses"],
        "budget_bytes": budget_bytes, "max_slots": max_slots,
        "service_s_by_mesh": {k: {"n": len(v), "mean": float(sum(v) / len(v))} for k, v in sorted(kinds.items())},
    }


def c3_batched_size():
    return (64, 32, 32), 64


def timed(fn, k=1):
    """Wall time of k calls of fn between two device synchronisations."""
    import torch
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    out = [fn() for _ in range(k)]
    torch.cuda.synchronize()
    return time.perf_counter() - t0, out


def headline_case(K, W, fp64_steps):
    """The metric's workload: one full hot-path iteration for 64 load cases
    per step, batched FP32 state solves with FP64 refinement, against the same
    step with plain FP64 solves."""
    import numpy as np
    import torch
    import fo_inputs as fi
    from paper_2601_05709_amd import fo
    from paper_2601_05709_amd.pipeline import Iteration
    cells, n_loads = c3_batched_size()
    w = fi.multi_load_3d(cells, n_loads, seed=3)
    m = w.mesh
    t0 = time.perf_counter()
    it = Iteration(w, fo.SolveOpts(precision=fo.FO_FP32_IR, rtol=1e-8),
                   fo.SolveOpts(precision=fo.FO_FP32_IR, rtol=1e-8), max_rhs=n_loads)
    it.ctx.set_levelset(it.phi0)
    log("c3: context in %.2f s" % (time.perf_counter() - t0))
    for _ in range(W):
        it.run()
    t_ir, outs = timed(lambda: it.run(update=True, reset_phi=True), K)
    st = outs[-1].state_stats
    log("c3: %.3f s/step (%.1f load-case solves/s), state %d block iterations + %d refinements, rel.res %.2e"
        % (t_ir / K, n_loads * K / t_ir, st.iters_inner, st.iters_outer, st.rel_res))
    u_ir = it.u.clone()
    rhs_ir = it.rhs.clone()
    it64 = Iteration(w, fo.SolveOpts(precision=fo.FO_FP64, rtol=1e-8), fo.SolveOpts(rtol=1e-8), max_rhs=n_loads)
    it64.run()
    t_64, outs64 = timed(lambda: it64.run(update=True, reset_phi=True), fp64_steps)
    st64 = outs64[-1].state_stats
    log("c3 plain FP64: %.3f s/step (%.1f load-case solves/s), %d iterations over the columns"
        % (t_64 / fp64_steps, n_loads * fp64_steps / t_64, st64.iters_inner))
    # accuracy: 8 columns against the GPU's FP64 CG at rel. res 1e-12 (that
    # solver matches the oracle in the parity tests)
    ref_cols = list(range(0, n_loads, n_loads // 8))
    bcol = it.b
    uref = torch.zeros(m.n_dofs, dtype=torch.float64, device="cuda")
    errs, errs64 = [], []
    for k in ref_cols:
        it64.ctx.state_solve(bcol[:, k].contiguous(), uref, fo.SolveOpts(precision=fo.FO_FP64, rtol=1e-12))
        nr = torch.linalg.norm(uref)
        errs.append(float(torch.linalg.norm(u_ir[:, k] - uref) / nr))
        errs64.append(float(torch.linalg.norm(it64.u[:, k] - uref) / nr))
    err_rhs = float(torch.linalg.norm(rhs_ir - it64.rhs) / torch.linalg.norm(it64.rhs))
    # the batched solves at rel. res 1e-9: the tolerance at which the
    # displacement error meets 1e-8 (a 1e-8 residual leaves errors up to a few
    # 1e-8 on this ill-conditioned operator)
    it.ctx.set_levelset(it.phi0)
    u9 = torch.zeros_like(it.u)
    o9 = fo.SolveOpts(precision=fo.FO_FP32_IR, rtol=1e-9)
    t_9, (s9,) = timed(lambda: it.ctx.state_solve(it.b, u9, o9, n_rhs=n_loads))
    errs9 = []
    for k in ref_cols:
        it64.ctx.state_solve(bcol[:, k].contiguous(), uref, fo.SolveOpts(precision=fo.FO_FP64, rtol=1e-12))
        errs9.append(float(torch.linalg.norm(u9[:, k] - uref) / torch.linalg.norm(uref)))
    # the state solves alone: batched, plain FP64 column by column, and the
    # single-load FP32 + refinement path column by column
    b = it.b
    u = torch.zeros_like(it.u)
    opts = fo.SolveOpts(precision=fo.FO_FP32_IR, rtol=1e-8)
    it.ctx.set_levelset(it.phi0)
    t_b, (sb,) = timed(lambda: it.ctx.state_solve(b, u, opts, n_rhs=n_loads))
    it.ctx.set_batch_method(fo.FO_BATCH_BLOCK_CG)
    bopts = fo.SolveOpts(precision=fo.FO_FP32_IR, rtol=1e-8, inner_rtol=1e-3)
    it.ctx.state_solve(b, u, bopts, n_rhs=n_loads)
    t_bcg, (sbcg,) = timed(lambda: it.ctx.state_solve(b, u, bopts, n_rhs=n_loads))
    it.ctx.set_batch_method(fo.FO_BATCH_COLUMN_CG)
    cols = [b[:, k].contiguous() for k in range(n_loads)]
    uc = torch.zeros(m.n_dofs, dtype=torch.float64, device="cuda")
    it.ctx.state_solve(cols[0], uc, opts)
    t_c, sc = timed(lambda: [it.ctx.state_solve(cols[k], uc, opts).iters_inner for k in range(n_loads)])
    its_c = sum(sc[0])
    apply_us = it.ctx.time_kernel(fo.FO_KERNEL_BATCH_APPLY, 50)
    # the element-tile operator on the same solves (tuned tiles), for comparison
    nodes, group, _ = it.ctx.batch_tune(n_loads)
    it.ctx.set_batch_operator(fo.FO_BATCH_OP_ELEMENT)
    el_apply_us = it.ctx.time_kernel(fo.FO_KERNEL_BATCH_APPLY, 20)
    it.ctx.state_solve(b, u, opts, n_rhs=n_loads)
    t_el, (sel,) = timed(lambda: it.ctx.state_solve(b, u, opts, n_rhs=n_loads))
    it.ctx.set_batch_operator(fo.FO_BATCH_OP_NODAL)
    d = m.dim
    width = 16 * ((n_loads + 15) // 16)
    ns = it.ctx.nodal_stats()
    # algorithmic work of the nodal apply: per off-diagonal block and column,
    # d^2 products and adds of y_i += K_ij (x_j - x_i); bytes: the blocks
    # (d^2 FP32 each) and neighbour ids, x read once, y written once
    flops = 2 * d * d * width * ns["off_diagonal_blocks"]
    abytes = ns["off_diagonal_blocks"] * (4 * d * d + 4) + 2 * m.n_dofs * width * 4
    state_s = sum(o.state_stats.seconds for o in outs)
    col_apps = sum(o.state_stats.iters_inner for o in outs) * n_loads
    state64_s = sum(o.state_stats.seconds for o in outs64)
    apps64 = sum(o.state_stats.iters_inner for o in outs64)
    traffic = recorded_traffic(BATCH_PROFILE, cells, BATCH_SOURCES)
    achieved = flops / (apply_us * 1e-6) / 1e12
    gbs = abytes / (apply_us * 1e-6) / 1e9
    roofline = {"bound": "hbm", "achieved": gbs, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": gbs / HBM_PEAK_GBS, "traffic": traffic,
                "label": "effective: the iteration's working set (about 260 MB) sits at the size of the 256 MB "
                         "Infinity Cache",
                "kernel": "k_nodal_apply<3,%d> (batched K(phi) P from the assembled node blocks on the matrix cores, "
                          "v_mfma_f32_4x4x1f32, %d columns)" % (width, width),
                "bytes_per_launch": abytes, "avg_us": apply_us, "reps": 50,
                "byte_count": "off-diagonal blocks (d^2 FP32) and their neighbour ids, x read once and y written "
                              "once (FP32, %d columns)" % width,
                "arithmetic_intensity": flops / abytes,
                "mfma_side": {"flops_per_launch": flops, "achieved_tflops": achieved, "peak_tflops": 157.3,
                              "frac": achieved / 157.3,
                              "flop_count": "2 d^2 per off-diagonal block and column (y_i += K_ij (x_j - x_i))"}}
    res = {
        "value": n_loads * K / t_ir, "ms_per_step": 1e3 * t_ir / K, "roofline": roofline,
        "config": {"workload": "3D cantilever %dx%dx%d cubes x 6 tets, %d load cases on one level set, one full "
                               "hot-path iteration per step (batched FP32 state solves on the matrix cores + FP64 "
                               "refinement to rel. res 1e-8, compliance per case, summed shape derivative, H1 descent "
                               "solve, level-set update)" % (cells + (n_loads,)),
                   "n_elems": m.n_elems, "n_nodes": m.n_nodes, "n_dofs": m.n_dofs, "n_loads": n_loads},
        "dof_iters_per_s": m.n_dofs * col_apps / state_s,
        "state_solve_ms": 1e3 * state_s / K,
        "state_iters": {"block": st.iters_inner, "refinements": st.iters_outer},
        "descent_iters": outs[-1].descent_stats.iters_inner,
        "fp64": {"what": "the same step with the 64 state solves and the descent solve in plain FP64 CG",
                 "solves_per_s": n_loads * fp64_steps / t_64, "ms_per_step": 1e3 * t_64 / fp64_steps,
                 "steps": fp64_steps, "dof_iters_per_s": m.n_dofs * apps64 / state64_s,
                 "state_solve_ms": 1e3 * state64_s / fp64_steps, "state_iters": st64.iters_inner},
        "speedup_vs_fp64": t_64 / fp64_steps / (t_ir / K),
        "accuracy": {"reference": "GPU FP64 CG to rel. res 1e-12 on 8 of the 64 columns",
                     "max_rel_err_u_batched": max(errs), "max_rel_err_u_fp64": max(errs64),
                     "target": 1e-8, "batched_meets_target": max(errs) <= 1e-8,
                     "rel_diff_rhs_batched_vs_fp64": err_rhs,
                     "at_rel_res_1e-9": {"solves_per_s": n_loads / t_9, "seconds": t_9, "block_iters": s9.iters_inner,
                                         "max_rel_err_u": max(errs9), "meets_target": max(errs9) <= 1e-8}},
        "solves_only": {"batched_s": t_b, "batched_solves_per_s": n_loads / t_b, "block_iters": sb.iters_inner,
                        "fp32_ir_columnwise_s": t_c, "fp32_ir_columnwise_solves_per_s": n_loads / t_c,
                        "fp32_ir_columnwise_mean_iters": its_c / n_loads,
                        "speedup_vs_fp32_ir_columnwise": t_c / t_b,
                        "block_cg": {"what": "the same 64 solves by block CG (phase target 1e-3)", "seconds": t_bcg,
                                     "solves_per_s": n_loads / t_bcg, "block_iters": sbcg.iters_inner,
                                     "refinements": sbcg.iters_outer},
                        "element_operator": {"what": "the same 64 solves (CG per column) on the element-tile operator "
                                                     "(K_e contraction per tile, tuned)", "seconds": t_el,
                                             "solves_per_s": n_loads / t_el, "block_iters": sel.iters_inner,
                                             "apply_us": el_apply_us, "tiles": {"node_cap": nodes, "group": group}}},
        "nodal_operator": ns,
    }
    log("c3: x%.2f over plain FP64 per step; state solves alone x%.2f over column-wise FP32+refinement, "
        "x%.2f over the element operator; max column error %.2e (FP64 %.2e); apply %.1f us = %.0f GB/s "
        "(element operator %.0f us)"
        % (res["speedup_vs_fp64"], t_c / t_b, t_el / t_b, max(errs), max(errs64), apply_us, gbs, el_apply_us))
    it.ctx.close()
    it64.ctx.close()
    return w, res


def phase_times(it):
    """One iteration with a device synchronisation after each phase."""
    import torch
    c = it.ctx
    out = {}
    it.phi.copy_(it.phi0)
    t, _ = timed(lambda: c.set_levelset(it.phi))
    out["levelset_ms"] = 1e3 * t
    t, (st,) = timed(lambda: c.state_solve(it.b, it.u, it.state_opts, n_rhs=it.n_rhs))
    out["state_ms"] = 1e3 * t
    t, _ = timed(lambda: c.shape_derivative(it.u, it.rhs, it.J, it.vol, n_rhs=it.n_rhs))
    out["derivative_ms"] = 1e3 * t
    t, (ds,) = timed(lambda: c.descent_solve(it.dopts, it.rhs, it.theta, it.descent_opts, it.B_tt))
    out["descent_ms"] = 1e3 * t
    from paper_2601_05709_amd import fo
    _, _, dt = fo.time_steps(float(it.B_tt.item()))
    t, _ = timed(lambda: c.levelset_update(it.theta, dt, it.phi))
    out["update_ms"] = 1e3 * t
    out["total_ms"] = sum(v for k, v in out.items() if k.endswith("_ms"))
    out["state_iters"] = {"inner": st.iters_inner, "outer": st.iters_outer}
    out["descent_iters"] = ds.iters_inner
    out["state_rel_res"] = st.rel_res
    return out


def paper_mesh_case():
    """The paper's 3D cantilever mesh size, 120x60x60 cubes x 6 tets (2.59M
    elements): one full iteration in FP32 + refinement and in plain FP64 with
    per-phase times (the second of each, after graph capture)."""
    import torch
    import fo_inputs as fi
    from paper_2601_05709_amd import fo
    from paper_2601_05709_amd.pipeline import Iteration
    cells = (120, 60, 60)
    w = fi.cantilever_3d(cells)
    m = w.mesh
    out = {"workload": "3D cantilever %dx%dx%d cubes x 6 tets (the paper's 3D mesh size), one load case, one full "
                       "hot-path iteration" % cells, "n_elems": m.n_elems, "n_nodes": m.n_nodes, "n_dofs": m.n_dofs}
    for key, prec in (("fp32_ir", fo.FO_FP32_IR), ("fp64", fo.FO_FP64)):
        it = Iteration(w, fo.SolveOpts(precision=prec, rtol=1e-8), fo.SolveOpts(precision=prec, rtol=1e-8))
        phase_times(it)
        out[key] = phase_times(it)
        if key == "fp32_ir":
            u_ir = it.u[:, 0].clone()
        else:
            out["err_u_fp32_ir_vs_fp64"] = float(torch.linalg.norm(u_ir - it.u[:, 0]) / torch.linalg.norm(it.u[:, 0]))
        it.ctx.close()
    log("c2 paper mesh %dx%dx%d: FP32+refinement %.1f ms per iteration (state %d + %d its), FP64 %.1f ms (%d its)"
        % (cells + (out["fp32_ir"]["total_ms"], out["fp32_ir"]["state_iters"]["inner"],
                    out["fp32_ir"]["state_iters"]["outer"], out["fp64"]["total_ms"],
                    out["fp64"]["state_iters"]["inner"])))
    return out


def large_case():
    """The large single instance, 256x128x128 cubes x 6 tets: one full
    iteration in FP32 + refinement and in plain FP64 with per-phase times, and
    the roofline of the fused CG operator where its working set exceeds the
    Infinity Cache (the HBM fraction is claimed here)."""
    import torch
    import fo_inputs as fi
    from paper_2601_05709_amd import fo
    from paper_2601_05709_amd.pipeline import Iteration
    cells = (256, 128, 128)
    t0 = time.perf_counter()
    w = fi.cantilever_3d(cells)
    m = w.mesh
    log("c5: mesh built in %.1f s (%d elements, %d unknowns)" % (time.perf_counter() - t0, m.n_elems, m.n_dofs))
    t0 = time.perf_counter()
    it = Iteration(w, fo.SolveOpts(precision=fo.FO_FP32_IR, rtol=1e-8),
                   fo.SolveOpts(precision=fo.FO_FP32_IR, rtol=1e-8))
    t_ctx = time.perf_counter() - t0
    log("c5: context in %.1f s (footprint %.2f GB)" % (t_ctx, it.ctx.footprint / 1e9))
    phase_times(it)  # warm-up (graph capture)
    ir = phase_times(it)
    log("c5 FP32+refinement: %.0f ms per iteration (state %.0f ms, %d + %d its)"
        % (ir["total_ms"], ir["state_ms"], ir["state_iters"]["inner"], ir["state_iters"]["outer"]))
    u_ir, rhs_ir = it.u[:, 0].clone(), it.rhs.clone()
    avg32 = it.ctx.time_kernel(fo.FO_KERNEL_CG_OP_FP32, 100)
    it64 = Iteration(w, fo.SolveOpts(precision=fo.FO_FP64, rtol=1e-8), fo.SolveOpts(rtol=1e-8))
    it.ctx.close()
    p64 = phase_times(it64)
    log("c5 FP64: %.0f ms per iteration (state %.0f ms, %d its)"
        % (p64["total_ms"], p64["state_ms"], p64["state_iters"]["inner"]))
    err_u = float(torch.linalg.norm(u_ir - it64.u[:, 0]) / torch.linalg.norm(it64.u[:, 0]))
    err_rhs = float(torch.linalg.norm(rhs_ir - it64.rhs) / torch.linalg.norm(it64.rhs))
    avg64 = it64.ctx.time_kernel(fo.FO_KERNEL_CG_OP_FP64, 100)
    it64.ctx.close()
    b32, b64 = fused_cg_bytes(m, 4), fused_cg_bytes(m, 8)
    a32 = b32 / (avg32 * 1e-6) / 1e9
    traffic = recorded_traffic(LARGE_PROFILE, cells, TRAFFIC_SOURCES)
    log("c5 roofline: fused FP32 CG operator %.1f us = %.0f GB/s (%.1f%% of HBM); FP64 %.1f us = %.0f GB/s"
        % (avg32, a32, 100 * a32 / HBM_PEAK_GBS, avg64, b64 / (avg64 * 1e-6) / 1e9))
    return {
        "workload": "3D cantilever %dx%dx%d cubes x 6 tets, one load case, one full hot-path iteration" % cells,
        "n_elems": m.n_elems, "n_nodes": m.n_nodes, "n_dofs": m.n_dofs, "context_s": t_ctx,
        "fp32_ir": ir, "fp64": p64, "err_u_fp32_ir_vs_fp64": err_u, "err_rhs_fp32_ir_vs_fp64": err_rhs,
        "error_vs_oracle": "on the 64x32x32 mesh (tests/test_gpu_large.py): the oracle's FP64 iteration is the "
                           "reference there",
        "roofline_hbm": {"bound": "hbm", "achieved": a32, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                         "frac": a32 / HBM_PEAK_GBS, "traffic": traffic,
                         "kernel": "k_tile_cg<3,float,ElasOp> (fused FP32 CG operator: direction update + tiled "
                                   "K(phi) apply)", "bytes_per_launch": b32, "avg_us": avg32, "reps": 100,
                         "fp64_avg_us": avg64, "fp64_bytes_per_launch": b64,
                         "fp64_achieved": b64 / (avg64 * 1e-6) / 1e9},
    }


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--cells", default="96,48,48", help="mesh of the single-load iteration (c2)")
    ap.add_argument("--fp64-steps", type=int, default=2, help="steps of the plain FP64 variant")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=20.0)
    ap.add_argument("--profile-only", action="store_true",
                    help="short run for profilers: the headline step only (one warm-up, one step)")
    ap.add_argument("--only", default=None, choices=["headline", "c2", "extras", "large", "paper"],
                    help="run one part alone (for profilers; extras: the single-load iteration and the "
                         "transport, reinitialisation, heat, inverse and loop measurements)")
    ap.add_argument("--kernel-only", default=None, choices=["headline", "large", "headline-solve"],
                    help="for counter passes: build the workload's context and time its dominant kernel only "
                         "(headline: the nodal batched apply on 64x32x32 with 64 columns; large: the fused FP32 CG "
                         "operator on 256x128x128), 20 launches; headline-solve: one warm-up and one timed batched "
                         "state solve of the 64 load cases (the iteration's kernels in their solve)")
    ap.add_argument("--no-large", action="store_true", help="skip the 256x128x128 instance")
    ap.add_argument("--main-only", action="store_true",
                    help="no transport, reinitialisation, heat, inverse or loop measurements")
    ap.add_argument("--no-serving", action="store_true", help="skip the serving stream")
    ap.add_argument("--serving-requests", type=int, default=120)
    args = ap.parse_args()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py measures one GPU only: the hot path is a single-GPU build "
              "(requested --gpus %d, WORLD_SIZE %d)" % (args.gpus, world), file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import fo_inputs as fi
    from paper_2601_05709_amd import fo
    from paper_2601_05709_amd.pipeline import Iteration

    torch.cuda.set_device(0)
    K = args.steps
    W = args.warmup
    if args.profile_only:
        K, W = 1, 1
    if args.only == "large":
        print(json.dumps(large_case()), flush=True)
        return
    if args.only == "paper":
        print(json.dumps(paper_mesh_case()), flush=True)
        return
    if args.kernel_only:
        if args.kernel_only == "headline-solve":
            cells, n_loads = c3_batched_size()
            wk = fi.multi_load_3d(cells, n_loads, seed=3)
            ctx = fo.Context.from_workload(wk, max_rhs=n_loads)
            ctx.set_levelset(torch.from_numpy(wk.phi).cuda())
            b = torch.from_numpy(wk.b).cuda()
            u = torch.zeros(wk.mesh.n_dofs, n_loads, dtype=torch.float64, device="cuda")
            opts = fo.SolveOpts(precision=fo.FO_FP32_IR, rtol=1e-8)
            ctx.state_solve(b, u, opts, n_rhs=n_loads)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            st = ctx.state_solve(b, u, opts, n_rhs=n_loads)
            torch.cuda.synchronize()
            print(json.dumps({"kernel_only": args.kernel_only, "solve_ms": 1e3 * (time.perf_counter() - t0),
                              "block_iters": st.iters_inner, "refinements": st.iters_outer,
                              "rel_res": st.rel_res}), flush=True)
            return
        if args.kernel_only == "headline":
            cells, n_loads = c3_batched_size()
            wk = fi.multi_load_3d(cells, n_loads, seed=3)
            ctx = fo.Context.from_workload(wk, max_rhs=n_loads)
            ctx.set_levelset(torch.from_numpy(wk.phi).cuda())
            us = ctx.time_kernel(fo.FO_KERNEL_BATCH_APPLY, 20)
        else:
            wk = fi.cantilever_3d((256, 128, 128))
            ctx = fo.Context.from_workload(wk)
            ctx.set_levelset(torch.from_numpy(wk.phi).cuda())
            us = ctx.time_kernel(fo.FO_KERNEL_CG_OP_FP32, 20)
        print(json.dumps({"kernel_only": args.kernel_only, "avg_us": us}), flush=True)
        return
    result = {"metric": "solves/s and DOF-iters/s at rel. res 1e-8: batched FP32+refine vs plain FP64",
              "value": None, "unit": "solves/s", "n_gpus": 1, "steps": K, "warmup": W, "ms_per_step": None,
              "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32+f64",
              "data": "synthetic"}
    w3 = None
    if args.only in (None, "headline"):
        log("headline: batched multi-load iteration, 64 loads on 64x32x32")
        w3, head = headline_case(K, W, 1 if args.profile_only else args.fp64_steps)
        result.update(head)
        if args.only == "headline" or args.profile_only:
            print(json.dumps(result), flush=True)
            return

    cells = tuple(int(c) for c in args.cells.split(","))
    log("c2: single-load workload %s" % (cells,))
    w = fi.cantilever_3d(cells)
    m = w.mesh
    t0 = time.perf_counter()
    it_ir = Iteration(w, fo.SolveOpts(precision=fo.FO_FP32_IR, rtol=1e-8),
                      fo.SolveOpts(precision=fo.FO_FP32_IR, rtol=1e-8))
    log("c2: context created in %.2f s (footprint %.1f MB, tiles %s)"
        % (time.perf_counter() - t0, it_ir.ctx.footprint / 1e6, it_ir.ctx.tile_stats()))
    it_64 = Iteration(w, fo.SolveOpts(precision=fo.FO_FP64, rtol=1e-8), fo.SolveOpts(rtol=1e-8))
    K2 = 5
    for _ in range(1):
        it_ir.run()
    t_ir, outs_ir = run_steps(it_ir, K2)
    st = outs_ir[-1].state_stats
    log("c2 FP32+refinement: %.3f s/step, state %d inner + %d outer its, rel.res %.2e"
        % (t_ir / K2, st.iters_inner, st.iters_outer, st.rel_res))
    it_64.run()
    t_64, outs_64 = run_steps(it_64, K2)
    st64 = outs_64[-1].state_stats
    log("c2 FP64: %.3f s/step, state %d its, rel.res %.2e" % (t_64 / K2, st64.iters_inner, st64.rel_res))
    if args.only == "c2":  # for profilers: the c2 iterations only
        print(json.dumps({"only": "c2", "ir_ms_per_step": 1e3 * t_ir / K2, "fp64_ms_per_step": 1e3 * t_64 / K2}),
              flush=True)
        return

    def extras():
        """The measurements besides the timed iteration: the paper's transport
        step and reinitialisation, the heat model and its loop, the inverse
        problem (one pair, its loop, eight pairs) and the compliance loop."""
        # the paper's transport step (Crank-Nicolson Petrov-Galerkin, BiCGStab)
        # with the velocity and adaptive final time of the last iteration, in
        # place of the one explicit update step of the timed iteration
        _, tr_steps, tr_dt = fo.time_steps(float(outs_ir[-1].B_tt.item()))
        phi_tr = it_ir.phi0.clone()
        it_ir.ctx.transport(it_ir.theta, tr_dt, tr_steps, phi_tr, fo.SolveOpts(rtol=1e-10))  # warm-up
        phi_tr.copy_(it_ir.phi0)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        st_tr = it_ir.ctx.transport(it_ir.theta, tr_dt, tr_steps, phi_tr, fo.SolveOpts(rtol=1e-10))
        torch.cuda.synchronize()
        t_tr = time.perf_counter() - t0
        log("transport step: %d Crank-Nicolson steps, %d BiCGStab operator applications, %.1f ms"
            % (tr_steps, st_tr.iters_inner, t_tr * 1e3))

        # the paper's reinitialisation (diffusive Eikonal, 8 steps to 0.1) of the
        # transported level set
        phi_rn = phi_tr.clone()
        it_ir.ctx.reinit(phi_rn, 8, 0.1, fo.SolveOpts(rtol=1e-10))  # warm-up
        phi_rn.copy_(phi_tr)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        st_rn = it_ir.ctx.reinit(phi_rn, 8, 0.1, fo.SolveOpts(rtol=1e-10))
        torch.cuda.synchronize()
        t_rn = time.perf_counter() - t0
        log("reinitialisation: 8 steps, %d BiCGStab operator applications, %.1f ms" % (st_rn.iters_inner, t_rn * 1e3))

        # the heat-conduction model on the same mesh (scalar P1 state, f = 1,
        # temperature fixed on the x = 0 face): load, state solve to rel. res
        # 1e-8, derivative, then the velocity solve as in the timed iteration
        f_ht = torch.ones(m.n_nodes, dtype=torch.float64, device="cuda")
        g0_ht = torch.from_numpy((np.abs(m.coords[:, 0]) < 1e-12).astype(np.uint8)).cuda()
        b_ht = torch.zeros_like(f_ht)
        u_ht = torch.zeros_like(f_ht)
        rhs_ht = torch.zeros(m.n_dofs, dtype=torch.float64, device="cuda")
        J_ht = torch.zeros(1, dtype=torch.float64, device="cuda")
        vol_ht = torch.zeros(1, dtype=torch.float64, device="cuda")
        th_ht = torch.zeros(m.n_dofs, dtype=torch.float64, device="cuda")
        Bt_ht = torch.zeros(1, dtype=torch.float64, device="cuda")
        it_ir.ctx.set_levelset(it_ir.phi0)

        def heat_step():
            it_ir.ctx.heat_load(f_ht, b_ht)
            s_ht = it_ir.ctx.heat_solve(g0_ht, b_ht, u_ht, fo.SolveOpts(rtol=1e-8))
            it_ir.ctx.heat_derivative(u_ht, f_ht, rhs_ht, J_ht, vol_ht)
            d_ht = it_ir.ctx.descent_solve(it_ir.dopts, rhs_ht, th_ht, fo.SolveOpts(precision=fo.FO_FP32_IR, rtol=1e-8),
                                           Bt_ht)
            return s_ht, d_ht

        heat_step()  # warm-up
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        st_ht, dst_ht = heat_step()
        torch.cuda.synchronize()
        t_ht = time.perf_counter() - t0
        log("heat model: state %d CG operator applications (%.1f ms), descent %d its, %.1f ms in all"
            % (st_ht.iters_inner, st_ht.seconds * 1e3, dst_ht.iters_inner, t_ht * 1e3))

        loop_iters = 4  # iterations of the timed loops (heat, inverse and compliance)

        # Algorithm 1 on the heat model (fo_optimize_heat): a few iterations with
        # the PPL volume constraint at 90% of the initial volume
        V_ht = 0.9 * float(vol_ht.item())
        phi_hl = it_ir.phi0.clone()
        it_ir.ctx.optimize_heat(g0_ht, f_ht, phi_hl, 1, it_ir.dopts, V=V_ht)  # warm-up
        phi_hl.copy_(it_ir.phi0)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        hl_recs, _ = it_ir.ctx.optimize_heat(g0_ht, f_ht, phi_hl, loop_iters, it_ir.dopts, V=V_ht)
        torch.cuda.synchronize()
        t_hl = time.perf_counter() - t0
        log("heat loop: %d iterations in %.3f s (%.1f ms per iteration), J %s"
            % (len(hl_recs), t_hl, 1e3 * t_hl / len(hl_recs), ["%.5g" % r["J"] for r in hl_recs]))

        # the paper's inverse elasticity problem (Kohn-Vogelius, kappa = 10) on a
        # mesh of the same size: states u, v and adjoints p, q (FP32 CG + FP64
        # refinement to rel. res 1e-8), cost, S0/S1 derivative and the H^1_0
        # velocity solve (every boundary unknown clamped)
        wi = fi.inverse_elasticity(cells)
        mi = wi.mesh
        t0 = time.perf_counter()
        inv_common = dict(E=wi.E, nu=wi.nu, plane_stress=wi.plane_stress, ersatz=1.0 / wi.kappa)
        cf_inv = fo.Context(mi.dim, mi.coords, mi.conn, wi.fixed0, mi.bfacets, mi.bnormal, **inv_common)
        # the second context on a stream of its own: its solves run concurrently with the first's
        side = torch.cuda.Stream()
        cg_inv = fo.Context(mi.dim, mi.coords, mi.conn, wi.fixed_all, None, None,
                            stream=fo.C.c_void_p(side.cuda_stream), **inv_common)
        log("inverse problem: two contexts created in %.2f s" % (time.perf_counter() - t0))

        def dvec(a, dtype=torch.float64):
            return torch.from_numpy(np.ascontiguousarray(a)).to(dtype).cuda()

        phi_inv, f_inv, g_inv = dvec(wi.phi), dvec(wi.f), dvec(wi.g)
        fx_inv = dvec(wi.fixed_all, torch.uint8)
        inv_out = [torch.zeros(mi.n_dofs, dtype=torch.float64, device="cuda") for _ in range(6)]
        u_iv, v_iv, p_iv, q_iv, rhs_iv, th_iv = inv_out
        J_iv = torch.zeros(1, dtype=torch.float64, device="cuda")
        Bt_iv = torch.zeros(1, dtype=torch.float64, device="cuda")
        dopts_iv = fo.DescentOpts(alpha=0.01, gamma_n=0.0, gamma_s=0.0, dim=3, fixed=fx_inv)

        def inverse_step():
            s_iv = cf_inv.inverse_states(cg_inv, phi_inv, f_inv, g_inv, wi.kappa, wi.alpha, wi.beta, u_iv, v_iv, p_iv,
                                         q_iv, J_iv, fo.SolveOpts(precision=fo.FO_FP32_IR, rtol=1e-8))
            cf_inv.inverse_derivative(u_iv, v_iv, p_iv, q_iv, g_inv, wi.kappa, wi.alpha, rhs_iv)
            d_iv = cf_inv.descent_solve(dopts_iv, rhs_iv, th_iv, fo.SolveOpts(precision=fo.FO_FP32_IR, rtol=1e-8), Bt_iv)
            return s_iv, d_iv

        inverse_step()  # warm-up
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        st_iv, dst_iv = inverse_step()
        torch.cuda.synchronize()
        t_iv = time.perf_counter() - t0
        log("inverse problem: 4 state solves %d + %d its (%.1f ms), velocity %d its, %.1f ms in all, J %.4g"
            % (st_iv.iters_inner, st_iv.iters_outer, st_iv.seconds * 1e3, dst_iv.iters_inner, t_iv * 1e3,
               float(J_iv.item())))

        # Algorithm 1 on the inverse problem (fo_optimize_inverse): a few
        # iterations from the initial inclusion, one pair
        phi_il = phi_inv.clone()
        cf_inv.optimize_inverse(cg_inv, f_inv, g_inv, wi.kappa, wi.alpha, wi.beta, phi_il, 1, dopts_iv)  # warm-up
        phi_il.copy_(phi_inv)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        il_recs, _ = cf_inv.optimize_inverse(cg_inv, f_inv, g_inv, wi.kappa, wi.alpha, wi.beta, phi_il, loop_iters,
                                             dopts_iv)
        torch.cuda.synchronize()
        t_il = time.perf_counter() - t0
        log("inverse loop: %d iterations in %.3f s (%.1f ms per iteration), J %s"
            % (len(il_recs), t_il, 1e3 * t_il / len(il_recs), ["%.5g" % r["J"] for r in il_recs]))
        cf_inv.close()
        cg_inv.close()

        # eight force-displacement pairs in one call (the cost and derivative
        # summed over the pairs), solved pair by pair
        npairs = 8
        wp = fi.inverse_elasticity(cells, n_pairs=npairs)
        cf_inv = fo.Context(mi.dim, mi.coords, mi.conn, wi.fixed0, mi.bfacets, mi.bnormal, **inv_common)
        cg_inv = fo.Context(mi.dim, mi.coords, mi.conn, wi.fixed_all, None, None,
                            stream=fo.C.c_void_p(side.cuda_stream), **inv_common)
        fP, gP = dvec(wp.columns(wp.fs)), dvec(wp.columns(wp.gs))
        uP, vP, pP, qP = (torch.zeros(mi.n_dofs * npairs, dtype=torch.float64, device="cuda") for _ in range(4))
        JP = torch.zeros(npairs, dtype=torch.float64, device="cuda")

        def inverse_pairs_step():
            s_p = cf_inv.inverse_states(cg_inv, phi_inv, fP, gP, wi.kappa, wi.alpha, wi.beta, uP, vP, pP, qP, JP,
                                        fo.SolveOpts(precision=fo.FO_FP32_IR, rtol=1e-8), n_pairs=npairs)
            cf_inv.inverse_derivative(uP, vP, pP, qP, gP, wi.kappa, wi.alpha, rhs_iv, n_pairs=npairs)
            d_p = cf_inv.descent_solve(dopts_iv, rhs_iv, th_iv, fo.SolveOpts(precision=fo.FO_FP32_IR, rtol=1e-8), Bt_iv)
            return s_p, d_p

        inverse_pairs_step()  # warm-up
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        st_ip, dst_ip = inverse_pairs_step()
        torch.cuda.synchronize()
        t_ip = time.perf_counter() - t0
        log("inverse problem, %d pairs: 4 x %d solves %d + %d its (%.1f ms), velocity %d its, %.1f ms in all "
            "(%.1f ms per pair)" % (npairs, npairs, st_ip.iters_inner, st_ip.iters_outer, st_ip.seconds * 1e3,
                                    dst_ip.iters_inner, t_ip * 1e3, t_ip * 1e3 / npairs))
        cf_inv.close()
        cg_inv.close()

        # the paper's loop (Algorithm 1, fo_optimize): a few iterations from the
        # initial design with the PPL volume constraint at 90% of its volume, the
        # paper's time-stepping defaults and transport step
        b_lp = it_ir.b[:, 0].contiguous()
        V_lp = 0.9 * float(outs_ir[-1].vol.item())
        phi_lp = it_ir.phi0.clone()
        it_ir.ctx.optimize(b_lp, phi_lp, 1, it_ir.dopts, V=V_lp)  # warm-up
        phi_lp.copy_(it_ir.phi0)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        lp_recs, _ = it_ir.ctx.optimize(b_lp, phi_lp, loop_iters, it_ir.dopts, V=V_lp)
        torch.cuda.synchronize()
        t_lp = time.perf_counter() - t0
        log("loop: %d iterations in %.3f s (%.1f ms per iteration, transport %s steps, lambda %s)"
            % (len(lp_recs), t_lp, 1e3 * t_lp / len(lp_recs), [r["steps"] for r in lp_recs],
               ["%.3g" % r["lambda"] for r in lp_recs]))

        return {
            "transport": {"what": "the paper's transport step (Crank-Nicolson Petrov-Galerkin, h^2 diffusion, "
                                  "FP64 Jacobi BiCGStab to rel. res 1e-10), not part of the timed iteration",
                          "ms": t_tr * 1e3, "steps": tr_steps, "dt": tr_dt,
                          "operator_applications": st_tr.iters_inner, "max_rel_res": st_tr.rel_res},
            "reinit": {"what": "the paper's reinitialisation (diffusive Eikonal, Petrov-Galerkin, explicit Euler then "
                               "Adams-Bashforth 2, 8 steps to pseudo-time 0.1, FP64 Jacobi BiCGStab to rel. res 1e-10) "
                               "of the transported level set, not part of the timed iteration",
                       "ms": t_rn * 1e3, "operator_applications": st_rn.iters_inner, "max_rel_res": st_rn.rel_res},
            "heat": {"what": "the paper's heat-conduction model on the same mesh (f = 1, u = 0 on x = 0): load, "
                             "FP64 state solve to rel. res 1e-8, S0/S1 derivative, FP32 + refinement velocity solve",
                     "ms": t_ht * 1e3, "state_ms": st_ht.seconds * 1e3, "state_operator_applications": st_ht.iters_inner,
                     "descent_iters": dst_ht.iters_inner, "J": float(J_ht.item()),
                     "loop": {"what": "Algorithm 1 on the heat model (fo_optimize_heat), PPL volume constraint at 90% "
                                      "of the initial volume", "iterations": len(hl_recs), "seconds": t_hl,
                              "ms_per_iteration": 1e3 * t_hl / len(hl_recs),
                              "records": [{k: r[k] for k in ("J", "C", "lambda", "steps", "state_iters",
                                                             "descent_iters", "transport_iters")} for r in hl_recs]}},
            "inverse": {"what": "the paper's inverse elasticity problem (kappa = 10, alpha = beta = 1) on a mesh of the "
                                "same size: u, v, p, q by FP32 CG + FP64 refinement to rel. res 1e-8, cost, S0/S1 "
                                "derivative, H^1_0 velocity solve", "ms": t_iv * 1e3, "states_ms": st_iv.seconds * 1e3,
                        "state_iters": {"inner_fp32": st_iv.iters_inner, "outer_fp64": st_iv.iters_outer},
                        "descent_iters": dst_iv.iters_inner, "J": float(J_iv.item()),
                        "pairs": {"what": "8 force-displacement pairs in one call: 4 x 8 solves by FP32 CG + FP64 "
                                          "refinement, derivative summed over the pairs, one velocity solve", "n_pairs": npairs, "ms": t_ip * 1e3, "ms_per_pair": t_ip * 1e3 / npairs,
                                  "states_ms": st_ip.seconds * 1e3,
                                  "state_iters": {"inner": st_ip.iters_inner, "outer": st_ip.iters_outer},
                                  "descent_iters": dst_ip.iters_inner},
                        "loop": {"what": "Algorithm 1 on the inverse problem (fo_optimize_inverse), one pair, from "
                                         "the initial inclusion", "iterations": len(il_recs), "seconds": t_il,
                                 "ms_per_iteration": 1e3 * t_il / len(il_recs),
                                 "records": [{k: r[k] for k in ("J", "steps", "state_iters", "descent_iters",
                                                                "transport_iters")} for r in il_recs]}},
            "loop": {"what": "the paper's Algorithm 1 (fo_optimize): state and velocity solves in FP32 + FP64 "
                             "refinement, PPL volume constraint at 90% of the initial volume, transport step, "
                             "from the initial design", "iterations": len(lp_recs), "seconds": t_lp,
                     "ms_per_iteration": 1e3 * t_lp / len(lp_recs),
                     "records": [{k: r[k] for k in ("J", "C", "lambda", "steps", "state_iters", "descent_iters",
                                                    "transport_iters")} for r in lp_recs]},
        }

    extra = {} if args.main_only else extras()
    if args.only == "extras":
        print(json.dumps({"only": "extras", **extra}), flush=True)
        return

    # agreement of the two precisions (both at rel. res 1e-8)
    u_ir = it_ir.u[:, 0].double()
    u_64 = it_64.u[:, 0].double()
    err_u = float(torch.linalg.norm(u_ir - u_64) / torch.linalg.norm(u_64))
    err_rhs = float(torch.linalg.norm(it_ir.rhs - it_64.rhs) / torch.linalg.norm(it_64.rhs))

    # the fused FP32 CG operator kernel k_tile_cg<3,float> on c2: average
    # duration inside one eager solve (an event pair around every launch) and
    # over back-to-back launches; the c2 working set stays in the Infinity
    # Cache, so the bandwidth is effective, not HBM
    ctx = it_ir.ctx
    ctx.profile_enable(True)
    it_ir.run()
    ms32, n32 = ctx.profile_read(fo.FO_PROF_ELAS_TILE_FP32)
    ctx.profile_enable(False)
    avg_solve_us = ms32 / max(n32, 1) * 1e3
    avg_us = ctx.time_kernel(fo.FO_KERNEL_CG_OP_FP32, 200)
    avg64_us = it_64.ctx.time_kernel(fo.FO_KERNEL_CG_OP_FP64, 200)
    bytes32 = fused_cg_bytes(m, 4)
    achieved = bytes32 / (avg_us * 1e-6) / 1e9
    log("c2 fused CG operator: %.1f us/launch back-to-back (%.1f in-solve), %.0f GB/s effective"
        % (avg_us, avg_solve_us, achieved))
    st_s = [o.state_stats for o in outs_ir]
    state_secs = sum(s_.seconds for s_ in st_s)
    state_its = sum(s_.iters_inner + s_.iters_outer for s_ in st_s)
    st64_s = [o.state_stats for o in outs_64]
    state64_secs = sum(s_.seconds for s_ in st64_s)
    state64_its = sum(s_.iters_inner for s_ in st64_s)
    result["c2"] = {
        "workload": "3D cantilever %dx%dx%d cubes x 6 tets, one load case, one full hot-path iteration per step "
                    "(FP32 CG + FP64 refinement to rel. res 1e-8)" % cells,
        "n_elems": m.n_elems, "n_nodes": m.n_nodes, "n_dofs": m.n_dofs, "steps": K2,
        "solves_per_s": K2 / t_ir, "ms_per_step": 1e3 * t_ir / K2,
        "dof_iters_per_s": m.n_dofs * state_its / state_secs,
        "state_iters": {"inner_fp32": st.iters_inner, "outer_fp64": st.iters_outer},
        "state_solve_ms": 1e3 * state_secs / K2,
        "descent_iters": outs_ir[-1].descent_stats.iters_inner,
        "fp64": {"solves_per_s": K2 / t_64, "ms_per_step": 1e3 * t_64 / K2,
                 "dof_iters_per_s": m.n_dofs * state64_its / state64_secs, "state_iters": st64.iters_inner,
                 "state_solve_ms": 1e3 * state64_secs / K2},
        "err_u_ir_vs_fp64": err_u, "err_rhs_ir_vs_fp64": err_rhs, "J": float(outs_ir[-1].J[0].item()),
        "roofline_effective": {"bound": "hbm", "label": "effective: the working set (about 50 MB) stays in the "
                               "256 MB Infinity Cache across iterations", "achieved": achieved,
                               "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS,
                               "traffic": recorded_traffic(TRAFFIC_PROFILE, cells, TRAFFIC_SOURCES),
                               "kernel": "k_tile_cg<3,float,ElasOp>", "bytes_per_launch": bytes32,
                               "avg_us": avg_us, "reps": 200, "avg_us_in_solve_event_pairs": avg_solve_us,
                               "launches_in_solve": n32, "fp64_avg_us": avg64_us,
                               "fp64_bytes_per_launch": fused_cg_bytes(m, 8),
                               "fp64_achieved": fused_cg_bytes(m, 8) / (avg64_us * 1e-6) / 1e9},
    }
    result.update(extra)
    it_ir.ctx.close()
    it_64.ctx.close()
    log("paper mesh size 120x60x60")
    result["c2_paper"] = paper_mesh_case()
    if not args.no_large:
        log("large instance 256x128x128")
        result["large"] = large_case()
    if not args.no_serving:
        log("serving stream (%d requests, 200/s)" % args.serving_requests)
        result["serving"] = serving_case(args.serving_requests)
        sv = result["serving"]
        log("serving: %.1f solves/s, latency p50 %.3f s p99 %.3f s" % (sv["solves_per_s"], sv["latency_p50_s"],
                                                                       sv["latency_p99_s"]))
    if not args.no_cpu and w3 is not None:
        log("CPU oracle baseline on the headline workload (~%.0f s)" % args.cpu_seconds)
        result["cpu_baseline"] = cpu_baseline_multi(w3, result["fp64"]["state_iters"] // w3.n_rhs,
                                                    result["descent_iters"], args.cpu_seconds)
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
