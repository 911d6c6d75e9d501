#!/usr/bin/env python3
"""Benchmark of the hot path on one MI355X.

Workload: the 3D cantilever box [0,2]x[0,1]^2 meshed with 96x48x48 cubes x 6
tetrahedra (1,327,104 elements, 232,897 nodes, 698,691 unknowns), 16 spherical
holes, clamp at x=0, unit -z traction on a 0.1x0.1 patch at the centre of the
face x=2.  A step is one full iteration of the hot path: level set ->
coefficients and Jacobi diagonal, state solve to relative residual 1e-8 (FP32
CG + FP64 iterative refinement), compliance and shape derivative, H1 descent
solve, explicit level-set update.  The same steps are also run with a plain
FP64 state solve for comparison.

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


# Kernel sources whose change invalidates recorded HBM traffic counters.
TRAFFIC_SOURCES = ["fo_tiled.hip", "fo_element.h", "fo_ops.h", "fo_reduce.h", "fo_internal.h",
                   "fo_tiles.cpp", "fo_tiles.h", "fo_xcd.h"]
TRAFFIC_PROFILE = os.path.join(ROOT, "profiles", "k_tile_cg_fp32_cantilever3d_96x48x48.md")


def kernel_source_hash():
    import hashlib
    h = hashlib.sha256()
    for f in TRAFFIC_SOURCES:
        with open(os.path.join(ROOT, "paper_2601_05709_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def recorded_traffic(path, cells):
    """HBM bytes per launch of the dominant kernel from the committed
    FETCH_SIZE/WRITE_SIZE counter summary, or None when the summary is
    missing, covers another mesh or was taken on other kernel sources."""
    try:
        fields = dict(line.split(":", 1) for line in open(path) if line.startswith("- ") and ":" in line)
    except OSError:
        return None
    fields = {k[2:].strip(): v.strip().strip("`") for k, v in fields.items()}
    if fields.get("source-sha256") != kernel_source_hash():
        return None
    if fields.get("cells") != "%dx%dx%d" % cells:
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


def cpu_baseline(w, iters_needed, descent_iters, budget_s):
    """The FP64 oracle on the host cores, one whole hot-path iteration on the
    same mesh: CSR assembly and Jacobi-PCG of the state, the shape
    derivative, the descent operator's assembly and Jacobi-PCG, the level-set
    update.  Each solve runs a bounded number of PCG iterations and is
    extrapolated to the iteration count the same algorithm (plain FP64
    Jacobi-PCG) needs on the GPU."""
    import numpy as np
    import oracle as oc
    m = w.mesh
    t0 = time.perf_counter()
    lam, mu = oc.lame(w.E, w.nu, m.dim, w.plane_stress)
    A, chi = oc.element_coef(m.dim, m.conn, w.phi, w.ersatz)
    K = oc.assemble_elasticity(m.dim, m.coords, m.conn, A, lam, mu)
    t_asm = time.perf_counter() - t0
    # rate probe long enough that the solve's set-up is a small part of it
    t0 = time.perf_counter()
    _, info = K.solve(w.b, w.fixed, rtol=1e-8, max_iter=100)
    t100 = time.perf_counter() - t0
    per = t100 / max(info.iters, 1)
    n = int(max(10, min(iters_needed, (0.6 * budget_s - t_asm) / max(per, 1e-9))))
    t0 = time.perf_counter()
    u, info = K.solve(w.b, w.fixed, rtol=1e-8, max_iter=n)
    t_it = time.perf_counter() - t0
    per = t_it / max(info.iters, 1)
    n_state = info.iters
    t0 = time.perf_counter()
    rhs, _, _, _ = oc.shape_derivative(m.dim, m.coords, m.conn, A, chi, lam, mu, u)
    t_sd = time.perf_counter() - t0
    t0 = time.perf_counter()
    B = oc.assemble_descent(m.dim, m.coords, m.conn, m.bfacets, m.bnormal, w.alpha, w.gamma_n, w.gamma_s, w.boxes)
    t_basm = time.perf_counter() - t0
    t0 = time.perf_counter()
    theta, dinfo = B.solve(rhs, None, rtol=1e-8, max_iter=max(10, int(descent_iters)))
    t_dit = time.perf_counter() - t0
    dper = t_dit / max(dinfo.iters, 1)
    t0 = time.perf_counter()
    oc.levelset_update(m.dim, m.coords, m.conn, theta, 1e-3, w.phi)
    t_up = time.perf_counter() - t0
    step_s = t_asm + iters_needed * per + t_sd + t_basm + descent_iters * dper + t_up
    return {
        "value": 1.0 / step_s,
        "unit": "solves/s",
        "cores": oc.get_threads(),
        "kind": "oracle",
        "sample": "one hot-path iteration on the same mesh: FP64 CSR assembly (%.2f s) + %d Jacobi-PCG "
                  "iterations of the state (%.2f s, extrapolated to the %d the same algorithm needs to reach "
                  "rel. res. 1e-8), shape derivative (%.2f s), descent assembly (%.2f s) + %d Jacobi-PCG "
                  "iterations (%.2f s, extrapolated to %d), level-set update (%.2f s)"
                  % (t_asm, n_state, t_it, iters_needed, t_sd, t_basm, dinfo.iters, t_dit, descent_iters, t_up),
        "dof_iters_per_s": m.n_dofs / per,
        "cpu_model": cpu_model(),
        "seconds_per_step": step_s,
        "assemble_s": t_asm,
        "s_per_iter": per,
    }


def batched_case(cells=(64, 32, 32), n_loads=64):
    """Batched multi-load solves: n_loads seeded load cases on one level set,
    FP32 matrix-core CG on all columns with FP64 residual replacement, against
    the same columns solved one after another in plain FP64 on the GPU."""
    import torch
    import fo_inputs as fi
    from paper_2601_05709_amd import fo
    w = fi.multi_load_3d(cells, n_loads, seed=3)
    m = w.mesh
    ctx = fo.Context.from_workload(w)
    ctx.set_levelset(torch.from_numpy(w.phi).cuda())
    nodes, group, _ = ctx.batch_tune(n_loads)
    b = torch.from_numpy(w.b).cuda()
    u = torch.zeros(m.n_dofs, n_loads, dtype=torch.float64, device="cuda")
    u64 = torch.zeros_like(u)
    opts = fo.SolveOpts(precision=fo.FO_FP32_IR, rtol=1e-8)
    ctx.state_solve(b, u, opts, n_rhs=n_loads)  # warm-up (graph capture)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    st = ctx.state_solve(b, u, opts, n_rhs=n_loads)
    torch.cuda.synchronize()
    t_b = time.perf_counter() - t0
    t0 = time.perf_counter()
    st64 = ctx.state_solve(b, u64, fo.SolveOpts(precision=fo.FO_FP64, rtol=1e-8), n_rhs=n_loads)
    torch.cuda.synchronize()
    t_64 = time.perf_counter() - t0
    # the same columns one after another on the single-load FP32 + refinement path
    cols = [b[:, k].contiguous() for k in range(n_loads)]
    uc = torch.zeros(m.n_dofs, dtype=torch.float64, device="cuda")
    ctx.state_solve(cols[0], uc, opts)
    torch.cuda.synchronize()
    its_c = 0
    t0 = time.perf_counter()
    for k in range(n_loads):
        its_c += ctx.state_solve(cols[k], uc, opts).iters_inner
    torch.cuda.synchronize()
    t_c = time.perf_counter() - t0
    err = float(((u - u64).norm(dim=0) / u64.norm(dim=0)).max())
    apply_us = ctx.time_kernel(fo.FO_KERNEL_BATCH_APPLY, 50)
    d = m.dim
    cols = 16 * ((n_loads + 15) // 16)
    flops = m.n_elems * cols * 2 * (d * (d + 1)) * (d * d)
    return {
        "workload": "3D cantilever %dx%dx%d cubes x 6 tets, %d load cases, rel. res 1e-8" % (cells + (n_loads,)),
        "solves_per_s": n_loads / t_b, "seconds": t_b, "block_iters": st.iters_inner,
        "max_replacements": st.iters_outer, "dof_iters_per_s": m.n_dofs * n_loads * st.iters_inner / t_b,
        "fp64_columnwise": {"solves_per_s": n_loads / t_64, "seconds": t_64, "iters": st64.iters_inner,
                            "dof_iters_per_s": m.n_dofs * st64.iters_inner / t_64},
        "speedup_vs_fp64_columnwise": t_64 / t_b,
        "fp32_ir_columnwise": {"solves_per_s": n_loads / t_c, "seconds": t_c, "mean_iters": its_c / n_loads},
        "speedup_vs_fp32_ir_columnwise": t_c / t_b,
        "max_col_rel_diff_vs_fp64": err,
        "tiles": {"node_cap": nodes, "group": group},
        "apply": {"kernel": "k_batch_apply<3,4,G> (FP32 MFMA 16x16x4, 64 columns)", "avg_us": apply_us,
                  "useful_flops": flops, "tflops": flops / (apply_us * 1e-6) / 1e12,
                  "peak_tflops_fp32_mfma": 157.3,
                  "frac": flops / (apply_us * 1e-6) / 1e12 / 157.3},
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


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--cells", default="96,48,48")
    ap.add_argument("--fp64-steps", type=int, default=None, help="steps of the plain FP64 variant")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=20.0)
    ap.add_argument("--profile-only", action="store_true", help="short run for profilers")
    ap.add_argument("--no-batched", action="store_true", help="skip the batched multi-load case")
    ap.add_argument("--main-only", action="store_true",
                    help="only the timed iteration, the precision check and the roofline (no transport, "
                         "reinitialisation, heat, inverse or loop measurements)")
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

    cells = tuple(int(c) for c in args.cells.split(","))
    log("building workload %s" % (cells,))
    w = fi.cantilever_3d(cells)
    m = w.mesh
    torch.cuda.set_device(0)
    t0 = time.perf_counter()
    it_ir = Iteration(w, fo.SolveOpts(precision=fo.FO_FP32_IR, rtol=1e-8),
                      fo.SolveOpts(precision=fo.FO_FP32_IR, rtol=1e-8))
    log("context created in %.2f s (footprint %.1f MB, tiles %s)"
        % (time.perf_counter() - t0, it_ir.ctx.footprint / 1e6, it_ir.ctx.tile_stats()))
    it_64 = Iteration(w, fo.SolveOpts(precision=fo.FO_FP64, rtol=1e-8), fo.SolveOpts(rtol=1e-8))

    K = 1 if args.profile_only else args.steps
    W = 0 if args.profile_only else args.warmup
    for _ in range(W):
        it_ir.run()
    log("warmup done; timing %d steps (FP32 CG + FP64 refinement)" % K)
    t_ir, outs_ir = run_steps(it_ir, K)
    st = outs_ir[-1].state_stats
    log("IR: %.3f s/step, state %d inner + %d outer its, rel.res %.2e"
        % (t_ir / K, st.iters_inner, st.iters_outer, st.rel_res))
    if args.profile_only:
        return

    K64 = args.fp64_steps if args.fp64_steps is not None else K
    it_64.run()
    t_64, outs_64 = run_steps(it_64, K64)
    st64 = outs_64[-1].state_stats
    log("FP64: %.3f s/step, state %d its, rel.res %.2e" % (t_64 / K64, st64.iters_inner, st64.rel_res))

    def extras():
        """The measurements besides the timed iteration: the paper's transport
        step and reinitialisation, the heat model and its loop, the inverse
        problem (one pair, its loop, eight pairs) and the compliance loop."""
        # the paper's transport step (Crank-Nicolson Petrov-Galerkin, BiCGStab)
        # with the velocity and adaptive final time of the last iteration, in
        # place of the one explicit update step of the timed iteration
        _, tr_steps, tr_dt = fo.adaptive_dt(float(outs_ir[-1].B_tt.item()))
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

    # agreement of the two precisions (both at rel. res 1e-8)
    u_ir = it_ir.u[:, 0].double()
    u_64 = it_64.u[:, 0].double()
    err_u = float(torch.linalg.norm(u_ir - u_64) / torch.linalg.norm(u_64))
    err_rhs = float(torch.linalg.norm(it_ir.rhs - it_64.rhs) / torch.linalg.norm(it_64.rhs))

    # roofline of the dominant kernel, the fused FP32 CG operator kernel
    # k_tile_cg<3,float>: its average duration inside one eager solve (a HIP
    # event pair around every launch) and over back-to-back launches (two
    # events around 200 launches, which is what a kernel profiler reports).
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
    traffic = recorded_traffic(TRAFFIC_PROFILE, cells)
    roofline = {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
                "kernel": "k_tile_cg<3,float,ElasOp> (fused FP32 CG operator: direction update + tiled K(phi) apply)",
                "bytes_per_launch": bytes32, "avg_us": avg_us, "reps": 200,
                "avg_us_in_solve_event_pairs": avg_solve_us, "launches_in_solve": n32,
                "fp64_avg_us": avg64_us, "fp64_bytes_per_launch": fused_cg_bytes(m, 8),
                "fp64_achieved": fused_cg_bytes(m, 8) / (avg64_us * 1e-6) / 1e9}
    log("roofline: %.1f us/launch back-to-back (%.1f in-solve with event pairs), %.0f GB/s (%.1f%% of HBM peak)"
        % (avg_us, avg_solve_us, achieved, 100 * achieved / HBM_PEAK_GBS))

    st_s = [o.state_stats for o in outs_ir]
    state_secs = sum(s.seconds for s in st_s)
    state_its = sum(s.iters_inner + s.iters_outer for s in st_s)
    st64_s = [o.state_stats for o in outs_64]
    state64_secs = sum(s.seconds for s in st64_s)
    state64_its = sum(s.iters_inner for s in st64_s)
    value = K / t_ir
    result = {
        "metric": "solves/s and DOF-iters/s at rel. res 1e-8: batched FP32+refine vs plain FP64",
        "value": value,
        "unit": "solves/s",
        "n_gpus": 1,
        "steps": K,
        "warmup": W,
        "ms_per_step": 1e3 * t_ir / K,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32+f64",
        "data": "synthetic",
        "config": {"workload": "3D cantilever %dx%dx%d cubes x 6 tets, FP32 CG + FP64 refinement to rel. res 1e-8, one full hot-path iteration per step" % cells,
                   "n_elems": m.n_elems, "n_nodes": m.n_nodes, "n_dofs": m.n_dofs},
        "dof_iters_per_s": m.n_dofs * state_its / state_secs,
        "state_iters": {"inner_fp32": st.iters_inner, "outer_fp64": st.iters_outer},
        "fp64": {"solves_per_s": K64 / t_64, "ms_per_step": 1e3 * t_64 / K64,
                 "dof_iters_per_s": m.n_dofs * state64_its / state64_secs,
                 "state_iters": st64.iters_inner,
                 "state_solve_ms": 1e3 * state64_secs / K64},
        "state_solve_ms": 1e3 * state_secs / K,
        "descent_iters": outs_ir[-1].descent_stats.iters_inner,
        "err_u_ir_vs_fp64": err_u,
        "err_rhs_ir_vs_fp64": err_rhs,
        "J": float(outs_ir[-1].J[0].item()),
        "roofline": roofline,
        "cpu_baseline": None,
    }
    result.update(extra)
    if not args.no_batched:
        log("batched multi-load case (64 loads, 64x32x32)")
        result["batched"] = batched_case()
        bt = result["batched"]
        log("batched: %.1f solves/s vs %.1f column-wise FP64 (x%.2f), %.1f column-wise FP32+refinement "
            "(x%.2f); apply %.0f us"
            % (bt["solves_per_s"], bt["fp64_columnwise"]["solves_per_s"], bt["speedup_vs_fp64_columnwise"],
               bt["fp32_ir_columnwise"]["solves_per_s"], bt["speedup_vs_fp32_ir_columnwise"],
               bt["apply"]["avg_us"]))
    if not args.no_serving:
        log("serving stream (%d requests, 200/s)" % args.serving_requests)
        result["serving"] = serving_case(args.serving_requests)
        sv = result["serving"]
        log("serving: %.1f solves/s, latency p50 %.3f s p99 %.3f s" % (sv["solves_per_s"], sv["latency_p50_s"],
                                                                       sv["latency_p99_s"]))
    if not args.no_cpu:
        log("CPU oracle baseline (~%.0f s)" % args.cpu_seconds)
        result["cpu_baseline"] = cpu_baseline(w, st64.iters_inner, outs_64[-1].descent_stats.iters_inner,
                                              args.cpu_seconds)
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
